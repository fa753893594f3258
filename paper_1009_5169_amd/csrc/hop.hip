// Wilson hopping term (half-dslash) for all right-hand sides of a block, with
// the epilogues that fuse it into D, D^+ and the CG vector updates, plus the
// finishing reduction and the CG vector kernels.
//
// H psi(n) = sum_mu [ (1 - g_mu) U_mu(n) psi(n+mu) + (1 + g_mu) U_mu(n-mu)^+ psi(n-mu) ]
// and its adjoint (projector signs swapped).  D = 1 - kappa H (Wilson quarks,
// Sections 3.1 and 4 of the paper; the operator itself is not written there).
// The even/odd split: the output parity p reads only the other parity, so
// H = H_eo + H_oe and one launch computes one of them for every RHS.
//
// Thread mapping: a workgroup is (sb sites) x (nr right-hand sides); a
// wavefront is 64 consecutive sites of one RHS, so every spinor and link load
// is a coalesced 16-, 8- or 4-byte-per-lane access and the nr wavefronts of a
// workgroup that read the same link tile hit in the CU's L1.
#include "internal.h"
#include "hop_impl.h"

namespace mfq {

// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8).  With remapping, XCD j walks the j-th contiguous chunk of site
// tiles, so the neighbour tiles a tile reads sit in the same XCD's L2.
__device__ __forceinline__ int tile_index(int remap) {
  const int nb = gridDim.x, b = blockIdx.x;
  if (!remap || nb < 16) return b;
  const int q = nb >> 3, rem = nb & 7, xcd = b & 7;
  return xcd * q + (xcd < rem ? xcd : rem) + (b >> 3);
}

// First half-lattice site of logical tile k (sb sites per tile).
template <typename S, typename SX>
__device__ __forceinline__ int tile_site0(const HopArgs<S, SX>& a, int k, int sb) {
  if (!a.zb) return k * sb;
  int rest = fdiv(k, a.mtpp);
  const int yt = k - rest * a.tpp;
  const int zi = rest & (a.zb - 1);
  rest >>= a.zbl;
  const int q = fdiv(rest, a.mtd);
  const int t = rest - q * a.g.td;
  const int z = q * a.zb + zi;
  return yt * sb + a.g.lxh * a.g.ly * (z + a.g.lz * t);
}

// The CG step length for RHS row `row`: from the scalars, or, when the
// |D p|^2 partials are passed (small lattices), reduced here by the row's
// leader wavefront in the same fixed order as the finishing kernel.  Split in
// two so that the partials' loads are issued at the start of the kernel and
// their latency hides behind the hopping term: alpha_fetch returns this
// lane's share, alpha_finish reduces it and broadcasts alpha through LDS (it
// holds a workgroup barrier).  On a breakdown (p^+ A p <= 0) alpha is 0 in
// every workgroup and workgroup 0 marks the RHS for a true-residual check.
template <typename S, typename SX>
__device__ __forceinline__ double alpha_fetch(const HopArgs<S, SX>& a, int r, bool leader) {
  double v = 0.0;
  if (a.apart && leader && r < a.n_rhs)
    for (int j = threadIdx.x; j < a.anblk; j += 64) v += a.apart[(long)r * a.anblk + j];
  return v;
}

template <typename S, typename SX>
__device__ __forceinline__ double alpha_finish(const HopArgs<S, SX>& a, int r, int row, bool leader, double v) {
  if (!a.apart) {
    __syncthreads();
    return r < a.n_rhs ? a.sc[r].alpha : 0.0;
  }
  __shared__ double s_alpha[8];
  if (leader) {
    v = wave_sum(v);
    if (threadIdx.x == 0) {
      double al = 0.0;
      if (r < a.n_rhs && a.sc[r].state == ST_ACTIVE) {
        if (isfinite(v) && v > 0.0) {
          al = a.sc[r].rho / v;
        } else if (blockIdx.x == 0) {
          a.sc[r].state = ST_CHECK;
        }
      }
      s_alpha[row] = al;
    }
  }
  __syncthreads();
  return s_alpha[row];
}

// With both parities in one launch (par == 2) consecutive tiles alternate
// parity over the same half-index range: the two tiles share the links of
// their rows (the forward link of one parity is the backward link of the
// other) and each other's spinors, so they meet in the same XCD's L2.
//
// With LDSL (FP32 / FP16 links) the workgroup first copies the 4 forward and
// 4 backward links of each of its sites into LDS, and every RHS row of the
// workgroup reads them from there: one link load serves all its RHS.
template <int EPI, typename S, typename SX, bool LDSL = false>
__global__ __launch_bounds__(512) void hop_kernel(HopArgs<S, SX> a) {
  const int tile = tile_index(a.xcd);
  int par = a.par;
  int s0;
  if (par == 2) {
    par = tile & 1;
    s0 = tile_site0(a, tile >> 1, blockDim.x);
  } else {
    s0 = tile_site0(a, tile, blockDim.x);
  }
  const int s = s0 + threadIdx.x;
  const int r = wave_uniform(blockIdx.y * blockDim.y + threadIdx.y);  // blockDim.x is a multiple of 64
  double av = 0.0;
  if constexpr (EPI == EPI_CGUPD) av = alpha_fetch(a, r, threadIdx.x < 64);
  bool active = s < a.g.vh && r < a.n_rhs;
  if (active && a.sc) active = a.upd_mode >= 0 ? in_update(a.sc[r], a.upd_mode) : a.sc[r].state < a.skip_state;
  using T = typename Compute<S>::T;
  Spinor<T> acc;
  zero(acc);
  if constexpr (LDSL) {
    using C = typename LinkChunk<S>::type;
    extern __shared__ __align__(16) unsigned char lds_link_tile[];
    C* tl = (C*)lds_link_tile;
    const int sb = blockDim.x;
    const C* gl = (const C*)a.links.data;
    // element e = lane + sb (chunk + 3 slot)
    for (int e = threadIdx.y * sb + threadIdx.x; e < 24 * sb; e += sb * blockDim.y) {
      const int lane = e % sb, k = (e / sb) % 3, slot = e / (3 * sb), mu = slot & 3;
      const int sl = s0 + lane;
      C v;
      v.x = v.y = v.z = v.w = 0;
      if (sl < a.g.vh) {
        if (slot < 4) {
          v = gl[a.links.cidx(par, mu, k, sl)];
        } else {
          const Coords cl = site_coords(a.g, sl, par);
          const int sbk = mu == 0   ? back_neighbour<0>(a.g, cl)
                          : mu == 1 ? back_neighbour<1>(a.g, cl)
                          : mu == 2 ? back_neighbour<2>(a.g, cl)
                                    : back_neighbour<3>(a.g, cl);
          v = gl[a.links.cidx(1 - par, mu, k, sbk)];
        }
      }
      tl[e] = v;
    }
    __syncthreads();
    if (active) hop_dirs_with<0, 4>(a, LdsLinks<S>{tl, sb, (int)threadIdx.x}, par, s, site_coords(a.g, s, par), r, acc);
  } else {
    if (active) hop_dirs<0, 4>(a, par, s, site_coords(a.g, s, par), r, acc);
  }
  double alpha = 0.0;
  if constexpr (EPI == EPI_CGUPD) alpha = alpha_finish(a, r, threadIdx.y, threadIdx.x < 64, av);
  const double red = active ? hop_epilogue<EPI>(a, par, s, r, alpha, acc) : 0.0;
  if (a.part) block_partial(red, a.part, a.n_rhs, blockIdx.y * blockDim.y, blockIdx.x, gridDim.x);
}

// Both parities, time sweep: workgroup tile = (time chunk, block of sb
// spatial sites); each thread walks the tc time slices of its spatial site, so
// the input it reads at t + 1 is its self term at t + 1 and its backward time
// neighbour at t + 2 (short reuse distances in the XCD's L2 instead of a whole
// time slice), and the threads of a wavefront cover consecutive x (both
// parities) of one time slice at every step.
template <int EPI, typename S, typename SX>
__global__ __launch_bounds__(512) void hop_sweep_kernel(HopArgs<S, SX> a, int tc, int nsb) {
  const int tile = tile_index(a.xcd);
  const int chunk = tile / nsb;
  const int sigma = (tile - chunk * nsb) * blockDim.x + threadIdx.x;
  const int r = wave_uniform(blockIdx.y * blockDim.y + threadIdx.y);  // blockDim.x is a multiple of 64
  const Geom& g = a.g;
  double alpha = 0.0;
  if constexpr (EPI == EPI_CGUPD)
    alpha = alpha_finish(a, r, threadIdx.y, threadIdx.x < 64, alpha_fetch(a, r, threadIdx.x < 64));
  bool active = sigma < g.lx * g.ly * g.lz && r < a.n_rhs;
  if (active && a.sc) active = a.upd_mode >= 0 ? in_update(a.sc[r], a.upd_mode) : a.sc[r].state < a.skip_state;
  double red = 0.0;
  if (active) {
    Coords c;
    c.x = sigma % g.lx;
    const int yz = sigma / g.lx;
    c.y = yz % g.ly;
    c.z = yz / g.ly;
    const int t0 = chunk * tc;
    const int t1 = t0 + tc < g.td ? t0 + tc : g.td;
    for (c.t = t0; c.t < t1; ++c.t) {
      const int par = (c.x + c.y + c.z + c.t + g.t0) & 1;
      red += hop_site<EPI, false>(a, par, half_index(g, c.x, c.y, c.z, c.t), c, r, alpha);  // par varies per lane
    }
  }
  if (a.part) block_partial(red, a.part, a.n_rhs, blockIdx.y * blockDim.y, blockIdx.x, gridDim.x);
}

// Direction split: a workgroup of DS x nr wavefronts covers 64 sites of nr
// RHS; wavefront w of a row computes directions [4w/DS, 4(w+1)/DS) of every
// site, the partial sums meet in LDS and the row's wavefront 0 applies the
// epilogue.  Each thread's chain of dependent loads is DS times shorter and a
// thread holds fewer registers, which is what bounds small lattices (one
// wavefront per CU or fewer) and helps latency hiding on large ones.
template <int EPI, int DS, typename S, typename SX>
__global__ __launch_bounds__(512) void hop_split_kernel(HopArgs<S, SX> a) {
  using T = typename Compute<S>::T;
  extern __shared__ __align__(16) unsigned char split_lds[];  // [rows][DS - 1][24][64] of T
  T(*lds)[DS - 1][24][64] = reinterpret_cast<T(*)[DS - 1][24][64]>(split_lds);
  const int tile = tile_index(a.xcd);
  int par = a.par;
  int s;
  if (par == 2) {
    par = tile & 1;
    s = tile_site0(a, tile >> 1, 64) + threadIdx.x;
  } else {
    s = tile_site0(a, tile, 64) + threadIdx.x;
  }
  const int ty = wave_uniform(threadIdx.y);  // blockDim.x is 64
  const int row = ty / DS, w = ty - row * DS;
  const int r = blockIdx.y * (blockDim.y / DS) + row;
  double av = 0.0;
  if constexpr (EPI == EPI_CGUPD) av = alpha_fetch(a, r, w == 0);
  bool active = s < a.g.vh && r < a.n_rhs;
  if (active && a.sc) active = a.upd_mode >= 0 ? in_update(a.sc[r], a.upd_mode) : a.sc[r].state < a.skip_state;
  Spinor<T> acc;
  zero(acc);
  if (active) {
    const Coords c = site_coords(a.g, s, par);
    if constexpr (DS == 2) {
      if (w == 0) hop_dirs<0, 2>(a, par, s, c, r, acc);
      else hop_dirs<2, 4>(a, par, s, c, r, acc);
    } else {
      if (w == 0) hop_dirs<0, 1>(a, par, s, c, r, acc);
      else if (w == 1) hop_dirs<1, 2>(a, par, s, c, r, acc);
      else if (w == 2) hop_dirs<2, 3>(a, par, s, c, r, acc);
      else hop_dirs<3, 4>(a, par, s, c, r, acc);
    }
  }
  if (w > 0) {
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      lds[row][w - 1][2 * k][threadIdx.x] = acc.v[k].re;
      lds[row][w - 1][2 * k + 1][threadIdx.x] = acc.v[k].im;
    }
  }
  // one barrier for the LDS partial terms and alpha
  double alpha = 0.0;
  if constexpr (EPI == EPI_CGUPD) alpha = alpha_finish(a, r, row, w == 0, av);
  else __syncthreads();
  if (w == 0) {
    double red = 0.0;
    if (active) {
#pragma unroll
      for (int q = 0; q < DS - 1; ++q)
#pragma unroll
        for (int k = 0; k < 12; ++k) {
          acc.v[k].re += lds[row][q][2 * k][threadIdx.x];
          acc.v[k].im += lds[row][q][2 * k + 1][threadIdx.x];
        }
      red = hop_epilogue<EPI>(a, par, s, r, alpha, acc);
    }
    if (a.part) {
      red = wave_sum(red);
      if (threadIdx.x == 0 && r < a.n_rhs) a.part[(long)r * gridDim.x + blockIdx.x] = red;
    }
  }
}

// RHS in the thread (order flag bit 3, FP32 / FP16 storage): each thread
// computes one site for R right-hand sides.  Every link is loaded and its
// third row rebuilt once per thread and applied to the R neighbour spinors,
// and the index arithmetic of each direction is shared by them, so a link
// load serves all R pseudo-fermions from registers rather than through the
// L1.  Groups of R RHS are grid.y; a ragged last group computes clamped
// copies of its last RHS and stores nothing for them.
template <int MU, int R, typename S, typename SX, typename T>
__device__ __forceinline__ void hop_dir_rt(const HopArgs<S, SX>& a, int par, const Coords& c, int s, const int (&rr)[R],
                                           T sgf, T sgb, Spinor<T> (&acc)[R]) {
  const int po = 1 - par;
  int sf, sbk;
  neighbours<MU>(a.g, c, s, sf, sbk);
  T wf, wb;
  time_factors<MU>(a.g, c, wf, wb);
  // 64-bit per-lane addresses here: a scalar buffer resource per RHS of the
  // group would exhaust the scalar registers.
  const PlainSrc<S, T> src{a.in};
  cpx<T> u[9];
  load_link(a.links, par, MU, s, u);
#pragma unroll
  for (int q = 0; q < R; ++q) {  // forward: (1 + sgf g_mu) U_mu(n) psi(n + mu)
    Spinor<T> nb;
    const T ns = src.load(rr[q], po, sf, nb);
    hop_half<MU, false, !std::is_same<S, _Float16>::value>(nb, u, sgf, wf * ns, acc[q]);
  }
  // keep the compiler from hoisting the next loads over this half: R
  // spinors in flight per half already cover the latency, more do not fit
  __builtin_amdgcn_sched_barrier(0);
  load_link(a.links, po, MU, sbk, u);
#pragma unroll
  for (int q = 0; q < R; ++q) {  // backward: U_mu(n - mu)^+ psi(n - mu)
    Spinor<T> nb;
    const T ns = src.load(rr[q], po, sbk, nb);
    hop_half<MU, true, !std::is_same<S, _Float16>::value>(nb, u, sgb, wb * ns, acc[q]);
  }
  __builtin_amdgcn_sched_barrier(0);
}

template <int EPI, int R, typename S, typename SX>
__global__ __launch_bounds__(256) void hop_rt_kernel(HopArgs<S, SX> a) {
  using T = typename Compute<S>::T;
  const int tile = tile_index(a.xcd);
  int par = a.par;
  int s0;
  if (par == 2) {
    par = tile & 1;
    s0 = tile_site0(a, tile >> 1, blockDim.x);
  } else {
    s0 = tile_site0(a, tile, blockDim.x);
  }
  const int s = s0 + threadIdx.x;
  const int r0 = blockIdx.y * R;
  int rr[R];
  bool live[R];
#pragma unroll
  for (int q = 0; q < R; ++q) {
    const int r = r0 + q;
    rr[q] = r < a.n_rhs ? r : a.n_rhs - 1;
    bool on = r < a.n_rhs;
    if (on && a.sc) on = a.upd_mode >= 0 ? in_update(a.sc[r], a.upd_mode) : a.sc[r].state < a.skip_state;
    live[q] = on;
  }
  // the fused CG step length: wave 0 reduces the |D p|^2 partials of every
  // RHS of the group (loads issued here, reduced after the hopping term)
  __shared__ double s_alpha[R];
  double av[R];
#pragma unroll
  for (int q = 0; q < R; ++q) av[q] = 0.0;
  if constexpr (EPI == EPI_CGUPD) {
    if (a.apart && threadIdx.x < 64)
#pragma unroll
      for (int q = 0; q < R; ++q)
        for (int j = threadIdx.x; j < a.anblk; j += 64) av[q] += a.apart[(long)rr[q] * a.anblk + j];
  }
  const bool site_ok = s < a.g.vh;
  Spinor<T> acc[R];
#pragma unroll
  for (int q = 0; q < R; ++q) zero(acc[q]);
  if (site_ok) {
    const Coords c = site_coords(a.g, s, par);
    const T sgf = a.dagger ? (T)1 : (T)-1;
    const T sgb = -sgf;
    hop_dir_rt<0, R>(a, par, c, s, rr, sgf, sgb, acc);
    hop_dir_rt<1, R>(a, par, c, s, rr, sgf, sgb, acc);
    hop_dir_rt<2, R>(a, par, c, s, rr, sgf, sgb, acc);
    hop_dir_rt<3, R>(a, par, c, s, rr, sgf, sgb, acc);
  }
  double alpha[R];
#pragma unroll
  for (int q = 0; q < R; ++q) alpha[q] = 0.0;
  if constexpr (EPI == EPI_CGUPD) {
    if (a.apart) {
      if (threadIdx.x < 64) {
#pragma unroll
        for (int q = 0; q < R; ++q) {
          const double v = wave_sum(av[q]);
          if (threadIdx.x == 0) {
            double al = 0.0;
            const int r = r0 + q;
            if (r < a.n_rhs && a.sc[r].state == ST_ACTIVE) {
              if (isfinite(v) && v > 0.0) al = a.sc[r].rho / v;
              else if (blockIdx.x == 0) a.sc[r].state = ST_CHECK;
            }
            s_alpha[q] = al;
          }
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < R; ++q) alpha[q] = s_alpha[q];
    } else {
#pragma unroll
      for (int q = 0; q < R; ++q) alpha[q] = r0 + q < a.n_rhs ? a.sc[r0 + q].alpha : 0.0;
    }
  }
  double red[R];
#pragma unroll
  for (int q = 0; q < R; ++q) red[q] = (site_ok && live[q]) ? hop_epilogue<EPI>(a, par, s, rr[q], alpha[q], acc[q]) : 0.0;
  if (a.part) {
    __shared__ double ws[R][4];
    const int wv = threadIdx.x >> 6;
#pragma unroll
    for (int q = 0; q < R; ++q) {
      const double v = wave_sum(red[q]);
      if ((threadIdx.x & 63) == 0) ws[q][wv] = v;
    }
    __syncthreads();
    if (threadIdx.x < R) {
      const int q = threadIdx.x;
      double t = 0.0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) t += ws[q][k];
      if (r0 + q < a.n_rhs) a.part[(long)(r0 + q) * gridDim.x + blockIdx.x] = t;
    }
  }
}

Shape default_shape(int n_rhs) {
  Shape sh;
  sh.xcd = 0;
  sh.tc = 0;
  sh.ds = 0;
  if (n_rhs <= 1) {
    sh.sb = 256;
    sh.nr = 1;
  } else if (n_rhs <= 2) {
    sh.sb = 128;
    sh.nr = 2;
  } else {
    sh.sb = 64;
    sh.nr = n_rhs < 8 ? n_rhs : 8;
  }
  return sh;
}

int hop_grid_x(const Geom& g, Shape sh, int par) {
  if (sh.ds > 1) sh.sb = 64;
  if (par == 2 && sh.tc > 0 && sh.ds <= 1)
    return ((g.lx * g.ly * g.lz + sh.sb - 1) / sh.sb) * ((g.td + sh.tc - 1) / sh.tc);
  const int per_parity = (g.vh + sh.sb - 1) / sh.sb;
  return par == 2 ? 2 * per_parity : per_parity;
}

int max_hop_blocks(const Geom& g) {
  int m = 2 * ((g.vh + 63) / 64);
  for (int tc = 2; tc <= 16; tc *= 2) {
    const int b = ((g.lx * g.ly * g.lz + 63) / 64) * ((g.td + tc - 1) / tc);
    if (b > m) m = b;
  }
  return m;
}

template <typename S, typename SX>
hipError_t launch_hop(int epi, const HopArgs<S, SX>& a, Shape sh, hipStream_t st) {
  HopArgs<S, SX> b = a;
  b.xcd = sh.xcd & 1;  // bit 1: z-blocked order (below); bit 2: LDS link tile (plain kernel); bit 3: RHS in the thread
  b.zb = 0;
  b.tpp = 0;
  {
    const int sbe = (sh.ds == 2 || sh.ds == 4) ? 64 : sh.sb;
    const int plane = a.g.lxh * a.g.ly;  // half sites per (z, t) plane
    if ((sh.xcd & 2) && (sh.tc == 0 || sh.ds > 1) && plane % sbe == 0) {
      b.zb = a.g.lz % 4 == 0 ? 4 : (a.g.lz % 2 == 0 ? 2 : 1);
      b.zbl = b.zb == 4 ? 2 : (b.zb == 2 ? 1 : 0);
      b.tpp = plane / sbe;
      b.mtpp = fdiv_magic(b.tpp);
      b.mtd = fdiv_magic(a.g.td);
    }
  }
  if (sh.ds == 2 || sh.ds == 4) {
    Shape s64 = sh;
    s64.sb = 64;
    s64.tc = 0;
    const dim3 grid(hop_grid_x(a.g, s64, a.par), (a.n_rhs + sh.nr - 1) / sh.nr), block(64, sh.ds * sh.nr);
    using T = typename Compute<S>::T;
    const size_t lds_bytes = (size_t)sh.nr * (sh.ds - 1) * 24 * 64 * sizeof(T);
#define MFQ_SPLIT(E)                                                                    \
  do {                                                                                  \
    if (sh.ds == 2)                                                                     \
      hipLaunchKernelGGL((hop_split_kernel<E, 2, S, SX>), grid, block, lds_bytes, st, b); \
    else                                                                                \
      hipLaunchKernelGGL((hop_split_kernel<E, 4, S, SX>), grid, block, lds_bytes, st, b); \
  } while (0)
    switch (epi) {
      case EPI_HOP: MFQ_SPLIT(EPI_HOP); break;
      case EPI_D: MFQ_SPLIT(EPI_D); break;
      case EPI_CGUPD: MFQ_SPLIT(EPI_CGUPD); break;
      case EPI_RES:
        if constexpr (sizeof(S) == 8) {
          MFQ_SPLIT(EPI_RES);
          break;
        }
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
#undef MFQ_SPLIT
    return hipGetLastError();
  }
  if constexpr (sizeof(S) != 8) {
    if ((sh.xcd & 8) && sh.tc == 0) {
      // RHS in the thread: sh.nr RHS per thread, sh.sb sites per workgroup
      const dim3 grid(hop_grid_x(a.g, sh, a.par), (a.n_rhs + sh.nr - 1) / sh.nr), block(sh.sb);
#define MFQ_RT(E, R) hipLaunchKernelGGL((hop_rt_kernel<E, R, S, SX>), grid, block, 0, st, b)
#define MFQ_RT_N(E)                    \
  switch (sh.nr) {                     \
    case 2: MFQ_RT(E, 2); break;       \
    case 3: MFQ_RT(E, 3); break;       \
    case 4: MFQ_RT(E, 4); break;       \
    case 5: MFQ_RT(E, 5); break;       \
    case 8: MFQ_RT(E, 8); break;       \
    default: return hipErrorInvalidValue; \
  }
      switch (epi) {
        case EPI_HOP: MFQ_RT_N(EPI_HOP); break;
        case EPI_D: MFQ_RT_N(EPI_D); break;
        case EPI_CGUPD: MFQ_RT_N(EPI_CGUPD); break;
        default: return hipErrorInvalidValue;
      }
#undef MFQ_RT_N
#undef MFQ_RT
      return hipGetLastError();
    }
  }
  dim3 block(sh.sb, sh.nr);
  dim3 grid(hop_grid_x(a.g, sh, a.par), (a.n_rhs + sh.nr - 1) / sh.nr);
  if (a.par == 2 && sh.tc > 0) {
    const int nsb = (a.g.lx * a.g.ly * a.g.lz + sh.sb - 1) / sh.sb;
    switch (epi) {
      case EPI_HOP: hipLaunchKernelGGL((hop_sweep_kernel<EPI_HOP, S, SX>), grid, block, 0, st, b, sh.tc, nsb); break;
      case EPI_D: hipLaunchKernelGGL((hop_sweep_kernel<EPI_D, S, SX>), grid, block, 0, st, b, sh.tc, nsb); break;
      case EPI_CGUPD:
        hipLaunchKernelGGL((hop_sweep_kernel<EPI_CGUPD, S, SX>), grid, block, 0, st, b, sh.tc, nsb);
        break;
      case EPI_RES:
        if constexpr (sizeof(S) == 8) {
          hipLaunchKernelGGL((hop_sweep_kernel<EPI_RES, S, SX>), grid, block, 0, st, b, sh.tc, nsb);
          break;
        }
        return hipErrorInvalidValue;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  if constexpr (sizeof(S) != 8) {
    // LDS link tile (order flag bit 2): 24 chunks per site
    const size_t lds_bytes = (size_t)24 * sh.sb * sizeof(typename LinkChunk<S>::type);
    if ((sh.xcd & 4) && lds_bytes <= 65536) {
      switch (epi) {
        case EPI_HOP: hipLaunchKernelGGL((hop_kernel<EPI_HOP, S, SX, true>), grid, block, lds_bytes, st, b); break;
        case EPI_D: hipLaunchKernelGGL((hop_kernel<EPI_D, S, SX, true>), grid, block, lds_bytes, st, b); break;
        case EPI_CGUPD:
          hipLaunchKernelGGL((hop_kernel<EPI_CGUPD, S, SX, true>), grid, block, lds_bytes, st, b);
          break;
        default: return hipErrorInvalidValue;
      }
      return hipGetLastError();
    }
  }
  switch (epi) {
    case EPI_HOP: hipLaunchKernelGGL((hop_kernel<EPI_HOP, S, SX>), grid, block, 0, st, b); break;
    case EPI_D: hipLaunchKernelGGL((hop_kernel<EPI_D, S, SX>), grid, block, 0, st, b); break;
    case EPI_CGUPD: hipLaunchKernelGGL((hop_kernel<EPI_CGUPD, S, SX>), grid, block, 0, st, b); break;
    case EPI_RES:
      if constexpr (sizeof(S) == 8) {
        hipLaunchKernelGGL((hop_kernel<EPI_RES, S, SX>), grid, block, 0, st, b);
        break;
      }
      return hipErrorInvalidValue;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template hipError_t launch_hop<double, double>(int, const HopArgs<double, double>&, Shape, hipStream_t);
template hipError_t launch_hop<float, float>(int, const HopArgs<float, float>&, Shape, hipStream_t);
template hipError_t launch_hop<_Float16, float>(int, const HopArgs<_Float16, float>&, Shape, hipStream_t);
template hipError_t launch_hop<_Float16, _Float16>(int, const HopArgs<_Float16, _Float16>&, Shape, hipStream_t);

// ------------------------------------------------------------ finishing
struct FinishArgs {
  Partials parts[4];
  int n_parts, n_rhs, fin;
  CgScalars* sc;
  double* out;
  double tol2, delta2;
};

__device__ void finish_apply(const FinishArgs& a, int r, double sum) {
  if (a.fin == FIN_STORE) {
    a.out[r] = sum;
    return;
  }
  cg_scalar_update(a.fin, a.sc[r], sum, a.tol2, a.delta2);
}

// Fixed-order reduction of the per-workgroup partials: deterministic, so FP64
// results are bitwise reproducible run to run.  One wavefront per RHS.
__global__ __launch_bounds__(1024) void finish_kernel(FinishArgs a) {
  const int lane = threadIdx.x & 63;
  for (int r = threadIdx.x >> 6; r < a.n_rhs; r += blockDim.x >> 6) {
    double v = 0.0;
    for (int q = 0; q < a.n_parts; ++q) {
      const double* p = a.parts[q].part + (long)r * a.parts[q].nblk;
      for (int j = lane; j < a.parts[q].nblk; j += 64) v += p[j];
    }
    v = wave_sum(v);
    if (lane == 0) finish_apply(a, r, v);
  }
}

hipError_t launch_finish(int fin, const Partials* parts, int n_parts, int n_rhs, CgScalars* sc,
                         double* out, double tol2, double delta2, hipStream_t st) {
  if (n_parts > 4) return hipErrorInvalidValue;
  FinishArgs a;
  for (int q = 0; q < n_parts; ++q) a.parts[q] = parts[q];
  a.n_parts = n_parts;
  a.n_rhs = n_rhs;
  a.fin = fin;
  a.sc = sc;
  a.out = out;
  a.tol2 = tol2;
  a.delta2 = delta2;
  const int waves = n_rhs < 16 ? (n_rhs > 0 ? n_rhs : 1) : 16;
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64 * waves), 0, st, a);
  return hipGetLastError();
}

// --------------------------------------------------------- vector kernels
// Lanes cover both parities (or the even one, npar = 1): q in [0, npar vh),
// parity q / vh, site q % vh.
#define MFQ_FULL_LANE                                             \
  const int q = blockIdx.x * blockDim.x + threadIdx.x;            \
  const int r = blockIdx.y * blockDim.y + threadIdx.y;            \
  if (q >= g.npar * g.vh || r >= n_rhs) return;                   \
  const int par = q >= g.vh ? 1 : 0;                              \
  const int s = q - par * g.vh;

template <typename S>
__global__ void xpay_p_kernel(Geom g, Field<S> rf, Field<S> pf, const CgScalars* sc, int n_rhs) {
  MFQ_FULL_LANE
  if (sc[r].state != ST_ACTIVE) return;
  using T = typename Compute<S>::T;
  const T beta = (T)sc[r].beta;
  Spinor<T> rr, pp;
  load_spinor(rf, r, par, s, rr);
  load_spinor(pf, r, par, s, pp);
#pragma unroll
  for (int k = 0; k < 12; ++k) pp.v[k] = rr.v[k] + beta * pp.v[k];
  store_spinor(pf, r, par, s, pp);
}

template <typename SX>
__global__ void fold_kernel(Geom g, Field<SX> xi, Field<double> x64, const CgScalars* sc, int n_rhs, int mode) {
  MFQ_FULL_LANE
  if (!in_update(sc[r], mode)) return;
  using TX = typename Compute<SX>::T;
  Spinor<TX> a;
  Spinor<double> b;
  load_spinor(xi, r, par, s, a);
  load_spinor(x64, r, par, s, b);
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    b.v[k].re += (double)a.v[k].re;
    b.v[k].im += (double)a.v[k].im;
    a.v[k] = {(TX)0, (TX)0};
  }
  store_spinor(x64, r, par, s, b);
  store_spinor(xi, r, par, s, a);
}

template <typename S>
__global__ void restart_kernel(Geom g, Field<double> r64, Field<S> ri, Field<S> pi, const CgScalars* sc,
                               int n_rhs) {
  MFQ_FULL_LANE
  if (sc[r].state != ST_ACTIVE || !sc[r].fresh) return;
  using T = typename Compute<S>::T;
  Spinor<double> a;
  load_spinor(r64, r, par, s, a);
  Spinor<T> b;
#pragma unroll
  for (int k = 0; k < 12; ++k) b.v[k] = {(T)a.v[k].re, (T)a.v[k].im};
  store_spinor(ri, r, par, s, b);
  const int rp = sc[r].rp;
  if (rp == 2) {
    const T beta = (T)sc[r].beta;
    Spinor<T> pp;
    load_spinor(pi, r, par, s, pp);
#pragma unroll
    for (int k = 0; k < 12; ++k) pp.v[k] = b.v[k] + beta * pp.v[k];
    store_spinor(pi, r, par, s, pp);
  } else if (rp == 1) {
    store_spinor(pi, r, par, s, b);
  }
}

template <typename SA, typename SB>
__global__ void convert_kernel(Geom g, Field<SA> src, Field<SB> dst, int gamma5, int n_rhs) {
  MFQ_FULL_LANE
  using TA = typename Compute<SA>::T;
  using TB = typename Compute<SB>::T;
  Spinor<TA> a;
  load_spinor(src, r, par, s, a);
  Spinor<TB> b;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const TB sg = (gamma5 && k >= 6) ? (TB)-1 : (TB)1;  // g5 = diag(1, 1, -1, -1)
    b.v[k] = {sg * (TB)a.v[k].re, sg * (TB)a.v[k].im};
  }
  store_spinor(dst, r, par, s, b);
}

__global__ void norm2_kernel(Geom g, Field<double> f, double* part, int n_rhs) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y * blockDim.y + threadIdx.y;
  double v = 0.0;
  if (q < g.npar * g.vh && r < n_rhs) {
    const int par = q >= g.vh ? 1 : 0;
    Spinor<double> a;
    load_spinor(f, r, par, q - par * g.vh, a);
    v = snorm2(a);
  }
  block_partial(v, part, n_rhs, blockIdx.y * blockDim.y, blockIdx.x, gridDim.x);
}

__global__ void init_residual_kernel(Geom g, Field<double> b, Field<double> r64, double* part, int n_rhs) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y * blockDim.y + threadIdx.y;
  double v = 0.0;
  if (q < g.npar * g.vh && r < n_rhs) {
    const int par = q >= g.vh ? 1 : 0;
    Spinor<double> a;
    load_spinor(b, r, par, q - par * g.vh, a);
    store_spinor(r64, r, par, q - par * g.vh, a);
    v = snorm2(a);
  }
  block_partial(v, part, n_rhs, blockIdx.y * blockDim.y, blockIdx.x, gridDim.x);
}

// A fixed nonzero test field (for kernel timing): component c of site q of
// RHS r holds a small integer hash mapped to [-0.5, 0.5).
__global__ void fill_pattern_kernel(Geom g, Field<double> f, int n_rhs) {
  MFQ_FULL_LANE
  Spinor<double> a;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const unsigned hsh = (unsigned)(q * 2654435761u) ^ (unsigned)(r * 40503u + k * 977u);
    a.v[k] = {(double)((hsh >> 8) & 1023) / 1024.0 - 0.5, (double)((hsh >> 18) & 1023) / 1024.0 - 0.5};
  }
  store_spinor(f, r, par, s, a);
}

template <typename S>
__global__ void zero_parity_kernel(Geom g, Field<S> f, int n_rhs, int par) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  if (s >= g.vh || r >= n_rhs) return;
  typename Store<S>::chunk z;
  for (int k = 0; k < (int)(sizeof(z) / sizeof(z[0])); ++k) z[k] = 0;
#pragma unroll
  for (int c = 0; c < Store<S>::NC; ++c) f.data[f.cidx(r, par, c, s)] = z;
  if constexpr (sizeof(S) == 2) f.norm[f.nidx(r, par, s)] = 0.f;
}

template <typename S>
hipError_t launch_zero_parity(const Geom& g, Field<S> f, int n_rhs, int par, hipStream_t st) {
  hipLaunchKernelGGL((zero_parity_kernel<S>), dim3((g.vh + 255) / 256, n_rhs), dim3(256), 0, st, g, f, n_rhs, par);
  return hipGetLastError();
}
template hipError_t launch_zero_parity<double>(const Geom&, Field<double>, int, int, hipStream_t);
template hipError_t launch_zero_parity<float>(const Geom&, Field<float>, int, int, hipStream_t);
template hipError_t launch_zero_parity<_Float16>(const Geom&, Field<_Float16>, int, int, hipStream_t);

static inline dim3 full_grid(const Geom& g, Shape sh, int n_rhs) {
  return dim3((g.npar * g.vh + sh.sb - 1) / sh.sb, (n_rhs + sh.nr - 1) / sh.nr);
}

template <typename S>
hipError_t launch_xpay_p(const Geom& g, Field<S> r, Field<S> p, const CgScalars* sc, int n_rhs,
                         Shape sh, hipStream_t st) {
  hipLaunchKernelGGL((xpay_p_kernel<S>), full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, r, p, sc, n_rhs);
  return hipGetLastError();
}
template <typename SX>
hipError_t launch_fold(const Geom& g, Field<SX> xi, Field<double> x64, const CgScalars* sc, int n_rhs, int mode,
                       Shape sh, hipStream_t st) {
  hipLaunchKernelGGL((fold_kernel<SX>), full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, xi, x64, sc, n_rhs,
                     mode);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_restart(const Geom& g, Field<double> r64, Field<S> ri, Field<S> pi, const CgScalars* sc,
                          int n_rhs, Shape sh, hipStream_t st) {
  hipLaunchKernelGGL((restart_kernel<S>), full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, r64, ri, pi, sc,
                     n_rhs);
  return hipGetLastError();
}
template <typename SA, typename SB>
hipError_t launch_convert(const Geom& g, Field<SA> src, Field<SB> dst, int gamma5, int n_rhs, Shape sh,
                          hipStream_t st) {
  hipLaunchKernelGGL((convert_kernel<SA, SB>), full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, src, dst,
                     gamma5, n_rhs);
  return hipGetLastError();
}
hipError_t launch_norm2(const Geom& g, Field<double> f, double* part, int n_rhs, Shape sh, int nblk,
                        hipStream_t st) {
  (void)nblk;
  hipLaunchKernelGGL(norm2_kernel, full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, f, part, n_rhs);
  return hipGetLastError();
}
hipError_t launch_fill_pattern(const Geom& g, Field<double> f, int n_rhs, Shape sh, hipStream_t st) {
  hipLaunchKernelGGL(fill_pattern_kernel, full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, f, n_rhs);
  return hipGetLastError();
}
hipError_t launch_init_residual(const Geom& g, Field<double> b, Field<double> r64, double* part, int n_rhs,
                                Shape sh, hipStream_t st) {
  hipLaunchKernelGGL(init_residual_kernel, full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, b, r64, part,
                     n_rhs);
  return hipGetLastError();
}

template hipError_t launch_xpay_p<double>(const Geom&, Field<double>, Field<double>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_xpay_p<float>(const Geom&, Field<float>, Field<float>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_xpay_p<_Float16>(const Geom&, Field<_Float16>, Field<_Float16>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_fold<double>(const Geom&, Field<double>, Field<double>, const CgScalars*, int, int, Shape, hipStream_t);
template hipError_t launch_fold<float>(const Geom&, Field<float>, Field<double>, const CgScalars*, int, int, Shape, hipStream_t);
template hipError_t launch_restart<double>(const Geom&, Field<double>, Field<double>, Field<double>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_restart<float>(const Geom&, Field<double>, Field<float>, Field<float>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_restart<_Float16>(const Geom&, Field<double>, Field<_Float16>, Field<_Float16>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_convert<double, double>(const Geom&, Field<double>, Field<double>, int, int, Shape, hipStream_t);
template hipError_t launch_convert<double, float>(const Geom&, Field<double>, Field<float>, int, int, Shape, hipStream_t);
template hipError_t launch_convert<double, _Float16>(const Geom&, Field<double>, Field<_Float16>, int, int, Shape, hipStream_t);
template hipError_t launch_convert<float, double>(const Geom&, Field<float>, Field<double>, int, int, Shape, hipStream_t);
template hipError_t launch_convert<_Float16, double>(const Geom&, Field<_Float16>, Field<double>, int, int, Shape, hipStream_t);

}  // namespace mfq
