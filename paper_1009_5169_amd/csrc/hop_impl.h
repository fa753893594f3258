// Device implementation of the Wilson hopping term and its fused epilogues,
// shared by the single-lattice kernels and the multi-lattice persistent
// kernels.
//
// H psi(n) = sum_mu [ (1 - g_mu) U_mu(n) psi(n+mu) + (1 + g_mu) U_mu(n-mu)^+ psi(n-mu) ]
// and its adjoint (projector signs swapped); D = 1 - kappa H.
#pragma once

#include <type_traits>

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

// Where the hopping term reads its input spinors.  load() returns the factor
// the spinor still has to be multiplied by: 1, or for FP16 storage the
// site's norm, which the hopping term folds into its accumulation.
template <typename S, typename T>
struct PlainSrc {
  Field<S> f;
  __device__ __forceinline__ T load(int r, int par, int s, Spinor<T>& o) const {
    load_spinor(f, r, par, s, o);
    return (T)1;
  }
};
template <typename T>
struct PlainSrc<_Float16, T> {
  Field<_Float16> f;
  __device__ __forceinline__ T load(int r, int par, int s, Spinor<T>& o) const {
    const float n = load_norm(f, r, par, s);
    load_spinor_raw(f, r, par, s, o);
    return (T)n;
  }
};

// The same through buffer resources: (r, par) uniform over the wavefront.
template <typename S, typename T>
struct BufSrc {
  Field<S> f;
  __device__ __forceinline__ T load(int r, int par, int s, Spinor<T>& o) const {
    buf_load_spinor(f, r, par, s, o);
    return (T)1;
  }
};
template <typename T>
struct BufSrc<_Float16, T> {
  Field<_Float16> f;
  __device__ __forceinline__ T load(int r, int par, int s, Spinor<T>& o) const {
    return (T)buf_load_spinor_raw(f, r, par, s, o);
  }
};

// A wave-uniform value (threadIdx.y of a workgroup whose x extent is a
// multiple of 64, anything derived from blockIdx) read into a scalar
// register, so that the addresses built from it stay scalar.
__device__ __forceinline__ int wave_uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

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

// The links through buffer resources (par uniform over the wavefront).
template <typename S>
struct BufLinks {
  Links<S> L;
  template <int MU, typename T>
  __device__ __forceinline__ void fwd(int par, int s, cpx<T> u[9]) const { buf_load_link(L, par, MU, s, u); }
  template <int MU, typename T>
  __device__ __forceinline__ void bwd(int po, int sbk, cpx<T> u[9]) const { buf_load_link(L, po, MU, sbk, u); }
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

// Half-lattice indices of the forward and backward neighbours of site s in
// direction MU: a step by the direction's stride, or the jump of a periodic
// wrap (the time boundary's factor is applied by the caller), from the
// site's coordinates without a multiply.  In x a step moves the half index
// only from an odd x forwards and from an even x backwards.
template <int MU>
__device__ __forceinline__ void neighbours(const Geom& g, const Coords& c, int s, int& sf, int& sb) {
  if constexpr (MU == 0) {
    sf = s + (c.t + 1 == g.td ? -g.wt : g.st);
    sb = s - (c.t == 0 ? -g.wt : g.st);
  } else if constexpr (MU == 1) {
    const bool odd = c.x & 1;
    sf = s + (odd ? (c.x + 1 == g.lx ? 1 - g.lxh : 1) : 0);
    sb = s - (odd ? 0 : (c.x == 0 ? 1 - g.lxh : 1));
  } else if constexpr (MU == 2) {
    sf = s + (c.y + 1 == g.ly ? -g.wy : g.sy);
    sb = s - (c.y == 0 ? -g.wy : g.sy);
  } else {
    sf = s + (c.z + 1 == g.lz ? -g.wz : g.sz);
    sb = s - (c.z == 0 ? -g.wz : g.sz);
  }
}

// o += a b and o += conj(a) b as chains of fused multiply-adds.
template <typename T>
__device__ __forceinline__ void cmac(cpx<T>& o, cpx<T> a, cpx<T> b) {
  o.re = fma(a.re, b.re, o.re);
  o.re = fma(-a.im, b.im, o.re);
  o.im = fma(a.re, b.im, o.im);
  o.im = fma(a.im, b.re, o.im);
}
template <typename T>
__device__ __forceinline__ void cjmac(cpx<T>& o, cpx<T> a, cpx<T> b) {
  o.re = fma(a.re, b.re, o.re);
  o.re = fma(a.im, b.im, o.re);
  o.im = fma(a.re, b.im, o.im);
  o.im = fma(-a.im, b.re, o.im);
}

// acc += w [g ; sg e_mu^+ g] for colour a, with sgw = sg w.
template <int MU, typename T>
__device__ __forceinline__ void reconstruct_w(Spinor<T>& acc, T w, T sgw, int a, cpx<T> g0, cpx<T> g1) {
  acc.v[a].re = fma(w, g0.re, acc.v[a].re);
  acc.v[a].im = fma(w, g0.im, acc.v[a].im);
  acc.v[3 + a].re = fma(w, g1.re, acc.v[3 + a].re);
  acc.v[3 + a].im = fma(w, g1.im, acc.v[3 + a].im);
  reconstruct_lower<MU>(acc, sgw, a, g0, g1);
}

// One half of direction MU: acc += w (1 + sg g_mu) V n with V = U (forward
// hop) or U^+ (backward hop, DAG): the projection to two spins, the colour
// multiply of both, and the accumulation into all four spins.  FUSED: the
// colour multiply as chains of fused multiply-adds and w folded into the
// accumulation.  For FP16 storage the compiler then keeps the half-precision
// operands packed for mixed-precision FMAs and runs out of registers, so
// FP16 takes the plain sums (FUSED = false).
template <int MU, bool DAG, bool FUSED, typename T>
__device__ __forceinline__ void hop_half(const Spinor<T>& n, const cpx<T> u[9], T sg, T w, Spinor<T>& acc) {
  cpx<T> h0[3], h1[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) project<MU>(n, sg, k, h0[k], h1[k]);
  if constexpr (!FUSED) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      cpx<T> g0, g1;
      if constexpr (!DAG) {
        g0 = cmul(u[3 * i], h0[0]) + cmul(u[3 * i + 1], h0[1]) + cmul(u[3 * i + 2], h0[2]);
        g1 = cmul(u[3 * i], h1[0]) + cmul(u[3 * i + 1], h1[1]) + cmul(u[3 * i + 2], h1[2]);
      } else {
        g0 = cjmul(u[i], h0[0]) + cjmul(u[3 + i], h0[1]) + cjmul(u[6 + i], h0[2]);
        g1 = cjmul(u[i], h1[0]) + cjmul(u[3 + i], h1[1]) + cjmul(u[6 + i], h1[2]);
      }
      reconstruct<MU>(acc, sg, i, w * g0, w * g1);
    }
    return;
  }
  const T sgw = sg * w;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    cpx<T> g0, g1;
    if constexpr (!DAG) {
      g0 = cmul(u[3 * i], h0[0]);
      g1 = cmul(u[3 * i], h1[0]);
      cmac(g0, u[3 * i + 1], h0[1]);
      cmac(g1, u[3 * i + 1], h1[1]);
      cmac(g0, u[3 * i + 2], h0[2]);
      cmac(g1, u[3 * i + 2], h1[2]);
    } else {  // (U^+)_{ik} = conj(U_{ki})
      g0 = cjmul(u[i], h0[0]);
      g1 = cjmul(u[i], h1[0]);
      cjmac(g0, u[3 + i], h0[1]);
      cjmac(g1, u[3 + i], h1[1]);
      cjmac(g0, u[6 + i], h0[2]);
      cjmac(g1, u[6 + i], h1[2]);
    }
    reconstruct_w<MU>(acc, w, sgw, i, g0, g1);
  }
}

// The factors of the forward and backward time hops: 1 inside, and across
// the time boundary 0 (Schroedinger functional: the neighbour is a boundary
// slice, outside the dynamical field), -1 (antiperiodic) or 1 (periodic).
template <int MU, typename T>
__device__ __forceinline__ void time_factors(const Geom& g, const Coords& c, T& wf, T& wb) {
  wf = (T)1;
  wb = (T)1;
  if constexpr (MU == 0) {
    const T wrap = g.bc == BC_SF ? (T)0 : (g.bc == BC_ANTIPERIODIC ? (T)-1 : (T)1);
    if (c.t + 1 == g.td) wf = wrap;
    if (c.t == 0) wb = wrap;
  }
}

// One direction mu of the hopping term: forward hop from n+mu through U_mu(n),
// backward hop from n-mu through U_mu(n-mu)^+.  sgf / sgb are the projector
// signs (-1 / +1 for H, +1 / -1 for H^+).  The time boundary is a factor on
// a neighbour index that always stays inside the lattice, so the loads of
// every direction are unconditional and can be issued together.
template <int MU, typename S, typename SX, typename T, typename Src, typename LS>
__device__ __forceinline__ void hop_dir(const HopArgs<S, SX>& a, const Src& src, const LS& lk, int par,
                                        const Coords& c, int s, int r, T sgf, T sgb, Spinor<T>& acc) {
  const int po = 1 - par;
  int sf, sbk;
  neighbours<MU>(a.g, c, s, sf, sbk);
  T wf, wb;
  time_factors<MU>(a.g, c, wf, wb);
  Spinor<T> nf, nb;
  cpx<T> uf[9], ub[9];
  const T nsf = src.load(r, po, sf, nf);
  lk.template fwd<MU>(par, s, uf);
  const T nsb = src.load(r, po, sbk, nb);
  lk.template bwd<MU>(po, sbk, ub);
  constexpr bool F = !std::is_same<S, _Float16>::value;
  hop_half<MU, false, F>(nf, uf, sgf, wf * nsf, acc);
  hop_half<MU, true, F>(nb, ub, sgb, wb * nsb, acc);
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
// UNI: r and par are uniform over the wavefront, so the spinors and links
// are read through scalar buffer resources; otherwise through 64-bit
// per-lane addresses.
template <int MU0, int MU1, bool UNI = true, typename S, typename SX, typename T, typename LS>
__device__ __forceinline__ void hop_dirs_with(const HopArgs<S, SX>& a, const LS& lk, int par, int s,
                                              const Coords& c, int r, Spinor<T>& acc) {
  const T sgf = a.dagger ? (T)1 : (T)-1;
  const T sgb = -sgf;
  using Src = typename std::conditional<UNI, BufSrc<S, T>, PlainSrc<S, T>>::type;
  const Src src{a.in};
  if constexpr (MU0 <= 0 && 0 < MU1) hop_dir<0>(a, src, lk, par, c, s, r, sgf, sgb, acc);
  if constexpr (MU0 <= 1 && 1 < MU1) hop_dir<1>(a, src, lk, par, c, s, r, sgf, sgb, acc);
  if constexpr (MU0 <= 2 && 2 < MU1) hop_dir<2>(a, src, lk, par, c, s, r, sgf, sgb, acc);
  if constexpr (MU0 <= 3 && 3 < MU1) hop_dir<3>(a, src, lk, par, c, s, r, sgf, sgb, acc);
}

template <int MU0, int MU1, bool UNI = true, typename S, typename SX, typename T>
__device__ __forceinline__ void hop_dirs(const HopArgs<S, SX>& a, int par, int s, const Coords& c, int r,
                                         Spinor<T>& acc) {
  if constexpr (UNI)
    hop_dirs_with<MU0, MU1, true>(a, BufLinks<S>{a.links}, par, s, c, r, acc);
  else
    hop_dirs_with<MU0, MU1, false>(a, GlobalLinks<S>{a.links}, par, s, c, r, acc);
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
template <int EPI, bool UNI = true, typename S, typename SX>
__device__ __forceinline__ double hop_site(const HopArgs<S, SX>& a, int par, int s, const Coords& c, int r,
                                           double al) {
  using T = typename Compute<S>::T;
  Spinor<T> acc;
  zero(acc);
  hop_dirs<0, 4, UNI>(a, par, s, c, r, acc);
  return hop_epilogue<EPI>(a, par, s, r, al, acc);
}

template <int EPI, typename S, typename SX>
__device__ __forceinline__ double hop_site(const HopArgs<S, SX>& a, int par, int s, int r, double al) {
  return hop_site<EPI>(a, par, s, site_coords(a.g, s, par), r, al);
}

}  // namespace mfq
