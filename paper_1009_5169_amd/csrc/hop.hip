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

// Partial sum of v over the sites of this workgroup, one value per RHS row.
__device__ __forceinline__ void block_partial(double v, double* part, int n_rhs) {
  __shared__ double ws[16];
  const int tid = threadIdx.y * blockDim.x + threadIdx.x;
  v = wave_sum(v);
  if ((tid & 63) == 0) ws[tid >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int wpr = blockDim.x >> 6;
    double s = 0.0;
    for (int k = 0; k < wpr; ++k) s += ws[threadIdx.y * wpr + k];
    const int r = blockIdx.y * blockDim.y + threadIdx.y;
    if (r < n_rhs) part[(long)r * gridDim.x + blockIdx.x] = s;
  }
}

// One direction mu of the hopping term: forward hop from n+mu through U_mu(n),
// backward hop from n-mu through U_mu(n-mu)^+.  sgf / sgb are the projector
// signs (-1 / +1 for H, +1 / -1 for H^+).
template <int MU, typename S, typename SX, typename T>
__device__ __forceinline__ void hop_dir(const HopArgs<S, SX>& a, const Coords& c, int s, int r,
                                        T sgf, T sgb, Spinor<T>& acc) {
  const Geom& g = a.g;
  const int po = 1 - a.par;
  {  // forward
    int x = c.x, y = c.y, z = c.z, t = c.t;
    T sgn = (T)1;
    bool ok = true;
    if constexpr (MU == 0) {
      t = c.t + 1;
      if (t == g.td) {
        if (g.bc == BC_SF) ok = false;
        t = 0;
        if (g.bc == BC_ANTIPERIODIC) sgn = (T)-1;
      }
    } else if constexpr (MU == 1) {
      x = (c.x + 1 == g.lx) ? 0 : c.x + 1;
    } else if constexpr (MU == 2) {
      y = (c.y + 1 == g.ly) ? 0 : c.y + 1;
    } else {
      z = (c.z + 1 == g.lz) ? 0 : c.z + 1;
    }
    if (ok) {
      Spinor<T> nb;
      load_spinor(a.in, r, po, half_index(g, x, y, z, t), nb);
      cpx<T> u[9];
      load_link(a.links, a.par, MU, s, u);
      cpx<T> h0[3], h1[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) project<MU>(nb, sgf, k, h0[k], h1[k]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        cpx<T> g0 = cmul(u[3 * i], h0[0]) + cmul(u[3 * i + 1], h0[1]) + cmul(u[3 * i + 2], h0[2]);
        cpx<T> g1 = cmul(u[3 * i], h1[0]) + cmul(u[3 * i + 1], h1[1]) + cmul(u[3 * i + 2], h1[2]);
        reconstruct<MU>(acc, sgf, i, sgn * g0, sgn * g1);
      }
    }
  }
  {  // backward
    int x = c.x, y = c.y, z = c.z, t = c.t;
    T sgn = (T)1;
    bool ok = true;
    if constexpr (MU == 0) {
      t = c.t - 1;
      if (t < 0) {
        if (g.bc == BC_SF) ok = false;
        t = g.td - 1;
        if (g.bc == BC_ANTIPERIODIC) sgn = (T)-1;
      }
    } else if constexpr (MU == 1) {
      x = (c.x == 0) ? g.lx - 1 : c.x - 1;
    } else if constexpr (MU == 2) {
      y = (c.y == 0) ? g.ly - 1 : c.y - 1;
    } else {
      z = (c.z == 0) ? g.lz - 1 : c.z - 1;
    }
    if (ok) {
      const int sb = half_index(g, x, y, z, t);
      Spinor<T> nb;
      load_spinor(a.in, r, po, sb, nb);
      cpx<T> u[9];
      load_link(a.links, po, MU, sb, u);
      cpx<T> h0[3], h1[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) project<MU>(nb, sgb, k, h0[k], h1[k]);
#pragma unroll
      for (int i = 0; i < 3; ++i) {  // (U^+)_{ik} = conj(U_{ki})
        cpx<T> g0 = cjmul(u[i], h0[0]) + cjmul(u[3 + i], h0[1]) + cjmul(u[6 + i], h0[2]);
        cpx<T> g1 = cjmul(u[i], h1[0]) + cjmul(u[3 + i], h1[1]) + cjmul(u[6 + i], h1[2]);
        reconstruct<MU>(acc, sgb, i, sgn * g0, sgn * g1);
      }
    }
  }
}

template <int EPI, typename S, typename SX>
__global__ __launch_bounds__(512) void hop_kernel(HopArgs<S, SX> a) {
  using T = typename Compute<S>::T;
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y * blockDim.y + threadIdx.y;
  bool active = s < a.g.vh && r < a.n_rhs;
  if (active && a.sc) active = a.sc[r].state < a.skip_state;
  double red = 0.0;
  if (active) {
    Spinor<T> acc;
    zero(acc);
    const Coords c = site_coords(a.g, s, a.par);
    const T sgf = a.dagger ? (T)1 : (T)-1;
    const T sgb = -sgf;
    hop_dir<0>(a, c, s, r, sgf, sgb, acc);
    hop_dir<1>(a, c, s, r, sgf, sgb, acc);
    hop_dir<2>(a, c, s, r, sgf, sgb, acc);
    hop_dir<3>(a, c, s, r, sgf, sgb, acc);
    const T b = (T)a.coef;
    if constexpr (EPI == EPI_HOP) {
#pragma unroll
      for (int k = 0; k < 12; ++k) acc.v[k] = b * acc.v[k];
      store_spinor(a.out, r, a.par, s, acc);
    } else if constexpr (EPI == EPI_D) {
      Spinor<T> self;
      load_spinor(a.self, r, a.par, s, self);
#pragma unroll
      for (int k = 0; k < 12; ++k) acc.v[k] = self.v[k] + b * acc.v[k];
      store_spinor(a.out, r, a.par, s, acc);
      red = snorm2(acc);
    } else if constexpr (EPI == EPI_CGUPD) {
      using TX = typename Compute<SX>::T;
      Spinor<T> self, rr, pp;
      Spinor<TX> xx;
      load_spinor(a.self, r, a.par, s, self);
      load_spinor(a.out, r, a.par, s, rr);
      load_spinor(a.p, r, a.par, s, pp);
      load_spinor(a.x, r, a.par, s, xx);
      const double al = a.sc[r].alpha;
      const T alpha = (T)al;
      const TX alx = (TX)al;
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cpx<T> ap = self.v[k] + b * acc.v[k];
        rr.v[k] = rr.v[k] - alpha * ap;
        xx.v[k] = xx.v[k] + alx * cpx<TX>{(TX)pp.v[k].re, (TX)pp.v[k].im};
      }
      store_spinor(a.out, r, a.par, s, rr);
      store_spinor(a.x, r, a.par, s, xx);
      red = snorm2(rr);
    } else {  // EPI_RES (FP64)
      Spinor<double> self, bb;
      load_spinor(a.self, r, a.par, s, self);
      load_spinor(a.bvec, r, a.par, s, bb);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cpx<double> ap = {(double)self.v[k].re + (double)b * (double)acc.v[k].re,
                                (double)self.v[k].im + (double)b * (double)acc.v[k].im};
        bb.v[k] = bb.v[k] - ap;
      }
      store_spinor(a.r64, r, a.par, s, bb);
      red = snorm2(bb);
    }
  }
  if (a.part) block_partial(red, a.part, a.n_rhs);
}

Shape default_shape(int n_rhs) {
  Shape sh;
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

int blocks_for(const Geom&, Shape sh, int n_sites) { return (n_sites + sh.sb - 1) / sh.sb; }

template <typename S, typename SX>
hipError_t launch_hop(int epi, const HopArgs<S, SX>& a, Shape sh, hipStream_t st) {
  dim3 block(sh.sb, sh.nr);
  dim3 grid((a.g.vh + sh.sb - 1) / sh.sb, (a.n_rhs + sh.nr - 1) / sh.nr);
  switch (epi) {
    case EPI_HOP: hipLaunchKernelGGL((hop_kernel<EPI_HOP, S, SX>), grid, block, 0, st, a); break;
    case EPI_D: hipLaunchKernelGGL((hop_kernel<EPI_D, S, SX>), grid, block, 0, st, a); break;
    case EPI_CGUPD: hipLaunchKernelGGL((hop_kernel<EPI_CGUPD, S, SX>), grid, block, 0, st, a); break;
    case EPI_RES:
      if constexpr (sizeof(S) == 8) {
        hipLaunchKernelGGL((hop_kernel<EPI_RES, S, SX>), grid, block, 0, st, a);
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
  CgScalars& s = a.sc[r];
  const bool finite = isfinite(sum);
  switch (a.fin) {
    case FIN_ALPHA:
      s.pap = sum;
      if (s.state == ST_ACTIVE && finite && sum > 0.0) {
        s.alpha = s.rho / sum;
      } else {
        if (s.state == ST_ACTIVE) s.state = ST_CHECK;  // breakdown: re-check truth
        s.alpha = 0.0;
      }
      break;
    case FIN_BETA:
      if (s.state == ST_ACTIVE) {
        s.beta = sum / s.rho;
        s.rho = sum;
        s.iters += 1;
        if (!finite || sum <= a.tol2 * s.bnorm2) s.state = ST_CHECK;
        if (sum < a.delta2 * s.rho_ru) s.upd = 1;
      } else {
        s.beta = 0.0;
      }
      break;
    case FIN_TRUE:
      if (s.state != ST_DONE) {
        s.rtrue2 = sum;
        s.n_true += 1;
        if (sum <= a.tol2 * s.bnorm2) {
          s.state = ST_DONE;
        } else {
          s.state = ST_ACTIVE;
          s.rho = sum;
          s.rho_ru = sum;
        }
        s.upd = 0;
      }
      break;
    case FIN_INIT:
      s.bnorm2 = sum;
      s.rho = s.rho_ru = s.rtrue2 = sum;
      s.alpha = s.beta = s.pap = 0.0;
      s.iters = s.upd = s.n_true = 0;
      s.state = sum > 0.0 ? ST_ACTIVE : ST_DONE;
      break;
  }
}

// Fixed-order reduction of the per-workgroup partials: deterministic, so FP64
// results are bitwise reproducible run to run.
__global__ __launch_bounds__(256) void finish_kernel(FinishArgs a) {
  __shared__ double ws[4];
  for (int r = 0; r < a.n_rhs; ++r) {
    double v = 0.0;
    for (int q = 0; q < a.n_parts; ++q) {
      const double* p = a.parts[q].part + (long)r * a.parts[q].nblk;
      for (int j = threadIdx.x; j < a.parts[q].nblk; j += 256) v += p[j];
    }
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) finish_apply(a, r, ((ws[0] + ws[1]) + ws[2]) + ws[3]);
    __syncthreads();
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
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, st, a);
  return hipGetLastError();
}

// --------------------------------------------------------- vector kernels
// Lanes cover both parities: q in [0, 2 vh), parity q / vh, site q % vh.
#define MFQ_FULL_LANE                                             \
  const int q = blockIdx.x * blockDim.x + threadIdx.x;            \
  const int r = blockIdx.y * blockDim.y + threadIdx.y;            \
  if (q >= 2 * g.vh || r >= n_rhs) return;                        \
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
__global__ void fold_kernel(Geom g, Field<SX> xi, Field<double> x64, const CgScalars* sc, int n_rhs) {
  MFQ_FULL_LANE
  if (sc[r].state == ST_DONE) return;
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
__global__ void restart_kernel(Geom g, Field<double> r64, Field<S> ri, Field<S> pi, int set_p,
                               const CgScalars* sc, int n_rhs) {
  MFQ_FULL_LANE
  if (sc[r].state != ST_ACTIVE) return;
  using T = typename Compute<S>::T;
  Spinor<double> a;
  load_spinor(r64, r, par, s, a);
  Spinor<T> b;
#pragma unroll
  for (int k = 0; k < 12; ++k) b.v[k] = {(T)a.v[k].re, (T)a.v[k].im};
  store_spinor(ri, r, par, s, b);
  if (set_p) store_spinor(pi, r, par, s, b);
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
  if (q < 2 * g.vh && r < n_rhs) {
    const int par = q >= g.vh ? 1 : 0;
    Spinor<double> a;
    load_spinor(f, r, par, q - par * g.vh, a);
    v = snorm2(a);
  }
  block_partial(v, part, n_rhs);
}

__global__ void init_residual_kernel(Geom g, Field<double> b, Field<double> r64, double* part, int n_rhs) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y * blockDim.y + threadIdx.y;
  double v = 0.0;
  if (q < 2 * g.vh && r < n_rhs) {
    const int par = q >= g.vh ? 1 : 0;
    Spinor<double> a;
    load_spinor(b, r, par, q - par * g.vh, a);
    store_spinor(r64, r, par, q - par * g.vh, a);
    v = snorm2(a);
  }
  block_partial(v, part, n_rhs);
}

static inline dim3 full_grid(const Geom& g, Shape sh, int n_rhs) {
  return dim3((2 * g.vh + sh.sb - 1) / sh.sb, (n_rhs + sh.nr - 1) / sh.nr);
}

template <typename S>
hipError_t launch_xpay_p(const Geom& g, Field<S> r, Field<S> p, const CgScalars* sc, int n_rhs,
                         Shape sh, hipStream_t st) {
  hipLaunchKernelGGL((xpay_p_kernel<S>), full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, r, p, sc, n_rhs);
  return hipGetLastError();
}
template <typename SX>
hipError_t launch_fold(const Geom& g, Field<SX> xi, Field<double> x64, const CgScalars* sc, int n_rhs,
                       Shape sh, hipStream_t st) {
  hipLaunchKernelGGL((fold_kernel<SX>), full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, xi, x64, sc, n_rhs);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_restart(const Geom& g, Field<double> r64, Field<S> ri, Field<S> pi, int set_p,
                          const CgScalars* sc, int n_rhs, Shape sh, hipStream_t st) {
  hipLaunchKernelGGL((restart_kernel<S>), full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, r64, ri, pi,
                     set_p, sc, n_rhs);
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
hipError_t launch_init_residual(const Geom& g, Field<double> b, Field<double> r64, double* part, int n_rhs,
                                Shape sh, hipStream_t st) {
  hipLaunchKernelGGL(init_residual_kernel, full_grid(g, sh, n_rhs), dim3(sh.sb, sh.nr), 0, st, g, b, r64, part,
                     n_rhs);
  return hipGetLastError();
}

template hipError_t launch_xpay_p<double>(const Geom&, Field<double>, Field<double>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_xpay_p<float>(const Geom&, Field<float>, Field<float>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_xpay_p<_Float16>(const Geom&, Field<_Float16>, Field<_Float16>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_fold<double>(const Geom&, Field<double>, Field<double>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_fold<float>(const Geom&, Field<float>, Field<double>, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_restart<double>(const Geom&, Field<double>, Field<double>, Field<double>, int, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_restart<float>(const Geom&, Field<double>, Field<float>, Field<float>, int, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_restart<_Float16>(const Geom&, Field<double>, Field<_Float16>, Field<_Float16>, int, const CgScalars*, int, Shape, hipStream_t);
template hipError_t launch_convert<double, double>(const Geom&, Field<double>, Field<double>, int, int, Shape, hipStream_t);
template hipError_t launch_convert<double, float>(const Geom&, Field<double>, Field<float>, int, int, Shape, hipStream_t);
template hipError_t launch_convert<double, _Float16>(const Geom&, Field<double>, Field<_Float16>, int, int, Shape, hipStream_t);
template hipError_t launch_convert<float, double>(const Geom&, Field<float>, Field<double>, int, int, Shape, hipStream_t);
template hipError_t launch_convert<_Float16, double>(const Geom&, Field<_Float16>, Field<double>, int, int, Shape, hipStream_t);

}  // namespace mfq
