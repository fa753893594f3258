// Canonical FP64 boundary layout <-> internal even/odd SoA layout, and the
// fermion MD force.
//
// Canonical spinor: [rhs][t][z][y][x][spin 4][colour 3] complex128 over the
// dynamical slices; canonical links and force: [mu][x0][z][y][x][3][3]
// complex128 over the stored link slices (x0 = 0..T for SF, 0..T-1 else).
#include <type_traits>

#include "internal.h"

namespace mfq {

template <typename S>
struct CT {
  using T = float;
};
template <>
struct CT<double> {
  using T = double;
};

__device__ __forceinline__ void canon_coords(const Geom& g, int q, int& x, int& y, int& z, int& t) {
  x = q % g.lx;
  int r = q / g.lx;
  y = r % g.ly;
  r /= g.ly;
  z = r % g.lz;
  t = r / g.lz;
}

template <typename S>
__global__ void pack_spinor_kernel(Geom g, const d2* canon, Field<S> f, int n_rhs, int gamma5, int* bad) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int vd = 2 * g.vh;
  if (q >= vd || r >= n_rhs) return;
  int x, y, z, t;
  canon_coords(g, q, x, y, z, t);
  const int par = (x + y + z + t + g.t0) & 1;
  const d2* src = canon + ((long)r * vd + q) * 12;
  using T = typename CT<S>::T;
  Spinor<T> o;
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    d2 v = src[k];
    finite = finite && isfinite(v.x) && isfinite(v.y);
    const double sg = (gamma5 && k >= 6) ? -1.0 : 1.0;
    o.v[k] = {(T)(sg * v.x), (T)(sg * v.y)};
  }
  if (!finite && bad) atomicOr(bad, 1);
  store_spinor(f, r, par, half_index(g, x, y, z, t), o);
}

__global__ void unpack_spinor_kernel(Geom g, Field<double> f, d2* canon, int n_rhs) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  const int vd = 2 * g.vh;
  if (q >= vd || r >= n_rhs) return;
  int x, y, z, t;
  canon_coords(g, q, x, y, z, t);
  const int par = (x + y + z + t + g.t0) & 1;
  Spinor<double> o;
  load_spinor(f, r, par, half_index(g, x, y, z, t), o);
  d2* dst = canon + ((long)r * vd + q) * 12;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    d2 v;
    v.x = o.v[k].re;
    v.y = o.v[k].im;
    dst[k] = v;
  }
}

// Links on the dynamical sites only: U_mu(n) for every dynamical n, mu.
// bad |= 1 for non-finite links; with su3_check, bad |= 2 for links that are
// not SU(3) to 1e-10 (|U U^+ - 1| or |det U - 1|), which rules out the
// two-row layout the FP32 / FP16 copies use (comp = 1 writes that layout).
template <typename S>
__global__ void pack_links_kernel(Geom g, const d2* canon, typename Store<S>::link_elem* out, int* bad, int comp,
                                  int su3_check) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int mu = blockIdx.y;
  const int vd = 2 * g.vh;
  if (q >= vd) return;
  int x, y, z, t;
  canon_coords(g, q, x, y, z, t);
  const int par = (x + y + z + t + g.t0) & 1;
  const int s = half_index(g, x, y, z, t);
  const long n_slice_sites = (long)g.lx * g.ly * g.lz;
  const int n_slices = g.td + (g.bc == BC_SF ? 2 : 0);
  const d2* src = canon + (((long)mu * n_slices + (t + g.t0)) * n_slice_sites + q % n_slice_sites) * 9;
  cpx<double> u[9];
  bool finite = true;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    d2 v = src[k];
    finite = finite && isfinite(v.x) && isfinite(v.y);
    u[k] = {v.x, v.y};
  }
  if (!finite && bad) atomicOr(bad, 1);
  if (su3_check && bad) {
    double dev = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        cpx<double> acc = {a == b ? -1.0 : 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 3; ++k) acc = acc + cjmul(u[3 * b + k], u[3 * a + k]);  // (U U^+)_ab - delta
        dev = fmax(dev, fabs(acc.re) + fabs(acc.im));
      }
    const cpx<double> det = cmul(u[0], cmul(u[4], u[8]) - cmul(u[5], u[7])) -
                            cmul(u[1], cmul(u[3], u[8]) - cmul(u[5], u[6])) +
                            cmul(u[2], cmul(u[3], u[7]) - cmul(u[4], u[6]));
    dev = fmax(dev, fabs(det.re - 1.0) + fabs(det.im));
    if (!(dev <= 1e-10)) atomicOr(bad, 2);
  }
  if constexpr (sizeof(S) != 8) {
    if (comp) {
      using C = typename std::conditional<sizeof(S) == 4, f4, h4>::type;
      C* co = (C*)out;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        C e;
        e.x = (S)u[2 * c].re;
        e.y = (S)u[2 * c].im;
        e.z = (S)u[2 * c + 1].re;
        e.w = (S)u[2 * c + 1].im;
        co[((long)(par * 4 + mu) * 3 + c) * g.vs + s] = e;
      }
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    typename Store<S>::link_elem e;
    e.x = (S)u[k].re;
    e.y = (S)u[k].im;
    out[((long)(par * 4 + mu) * 9 + k) * g.vs + s] = e;
  }
}

template <typename S>
hipError_t launch_pack_spinor(const Geom& g, const double* canon, Field<S> f, int n_rhs, int gamma5, int* bad,
                              hipStream_t st) {
  dim3 grid((2 * g.vh + 255) / 256, n_rhs);
  hipLaunchKernelGGL((pack_spinor_kernel<S>), grid, dim3(256), 0, st, g, (const d2*)canon, f, n_rhs, gamma5, bad);
  return hipGetLastError();
}
hipError_t launch_unpack_spinor(const Geom& g, Field<double> f, double* canon, int n_rhs, hipStream_t st) {
  dim3 grid((2 * g.vh + 255) / 256, n_rhs);
  hipLaunchKernelGGL(unpack_spinor_kernel, grid, dim3(256), 0, st, g, f, (d2*)canon, n_rhs);
  return hipGetLastError();
}
template <typename S>
hipError_t launch_pack_links(const Geom& g, const double* canon, typename Store<S>::link_elem* out, int* bad,
                             int comp, int su3_check, hipStream_t st) {
  dim3 grid((2 * g.vh + 255) / 256, 4);
  hipLaunchKernelGGL((pack_links_kernel<S>), grid, dim3(256), 0, st, g, (const d2*)canon, out, bad, comp, su3_check);
  return hipGetLastError();
}

template hipError_t launch_pack_spinor<double>(const Geom&, const double*, Field<double>, int, int, int*, hipStream_t);
template hipError_t launch_pack_spinor<float>(const Geom&, const double*, Field<float>, int, int, int*, hipStream_t);
template hipError_t launch_pack_spinor<_Float16>(const Geom&, const double*, Field<_Float16>, int, int, int*, hipStream_t);
template hipError_t launch_pack_links<double>(const Geom&, const double*, d2*, int*, int, int, hipStream_t);
template hipError_t launch_pack_links<float>(const Geom&, const double*, f2*, int*, int, int, hipStream_t);
template hipError_t launch_pack_links<_Float16>(const Geom&, const double*, h2*, int*, int, int, hipStream_t);

// ------------------------------------------------------------------ force
// For the link (n, mu), with X = D^-1 phi and Y = (D^+)^-1 X per RHS i:
//   A = sum_i sum_b h-[X_i(n+mu)]_b h-[Y_i(n)]_b^+ ,  h-[psi] = psi_up - e_mu psi_down
//   B = sum_i sum_b h+[X_i(n)]_b h+[Y_i(n+mu)]_b^+ ,  h+[psi] = psi_up + e_mu psi_down
//   M = U A - B U^+,   G = -kappa ( (M - M^+)/(2i) - Tr(...)/3 )
// which is Eq. 3's f[x_i, y_i] summed over i, with the RHS sum taken before
// the projection (the force is linear in the outer products).
//
// One thread per (link, half, RHS group): a workgroup is 64 sites x 2 NR
// threads; thread y takes the half y % 2 (U A or -B U^+) for the RHS
// y / 2, y / 2 + NR, ...; each forms its partial M, the partials meet in LDS
// and thread y = 0 of each site adds them in y order (a fixed order, so FP64
// results repeat bitwise), projects and stores.  Splitting the halves over
// threads halves each thread's registers (twice the resident wavefronts).
template <int MU>
__device__ __forceinline__ void force_partial(const Geom& g, const Links<double>& L, const Field<double>& X,
                                              const Field<double>& Y, int half, int r0, int n_rhs, int rstep, int par,
                                              int s, const Coords& c, bool& ok, double& sgn, cpx<double> M[9]) {
  int x = c.x, y = c.y, z = c.z, t = c.t;
  sgn = 1.0;
  ok = true;
  if constexpr (MU == 0) {
    t = c.t + 1;
    if (t == g.td) {
      if (g.bc == BC_SF) ok = false;
      t = 0;
      if (g.bc == BC_ANTIPERIODIC) sgn = -1.0;
    }
  } else if constexpr (MU == 1) {
    x = (c.x + 1 == g.lx) ? 0 : c.x + 1;
  } else if constexpr (MU == 2) {
    y = (c.y + 1 == g.ly) ? 0 : c.y + 1;
  } else {
    z = (c.z + 1 == g.lz) ? 0 : c.z + 1;
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) M[k] = {0.0, 0.0};
  if (!ok || r0 >= n_rhs) return;
  const int sf = half_index(g, x, y, z, t);
  const int po = 1 - par;
  // half 0: A from X(n + mu), Y(n) with h-; half 1: B from X(n), Y(n + mu) with h+
  const double sg = half == 0 ? -1.0 : 1.0;
  const int xp = half == 0 ? po : par, xs_site = half == 0 ? sf : s;
  const int yp = half == 0 ? par : po, ys_site = half == 0 ? s : sf;
  cpx<double> AB[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) AB[k] = {0.0, 0.0};
  for (int r = r0; r < n_rhs; r += rstep) {
    // colour by colour: the four spin components of colour k, projected at
    // once, so only the half spinors stay in registers
    cpx<double> hx0[3], hx1[3], hy0[3], hy1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Spinor<double> xs, ys;  // only components 3 sp + k are filled
#pragma unroll
      for (int sp = 0; sp < 4; ++sp) {
        const d2 qx = X.data[X.cidx(r, xp, 3 * sp + k, xs_site)];
        const d2 qy = Y.data[Y.cidx(r, yp, 3 * sp + k, ys_site)];
        xs.v[3 * sp + k] = {qx.x, qx.y};
        ys.v[3 * sp + k] = {qy.x, qy.y};
      }
      project<MU>(xs, sg, k, hx0[k], hx1[k]);
      project<MU>(ys, sg, k, hy0[k], hy1[k]);
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b)
        AB[3 * a + b] = AB[3 * a + b] + cjmul(hy0[b], hx0[a]) + cjmul(hy1[b], hx1[a]);
  }
  cpx<double> u[9];
  load_link(L, par, MU, s, u);
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cpx<double> m = {0.0, 0.0};
      if (half == 0) {
#pragma unroll
        for (int k = 0; k < 3; ++k) m = m + cmul(u[3 * a + k], AB[3 * k + b]);  // (U A)_{ab}
      } else {
#pragma unroll
        for (int k = 0; k < 3; ++k) m = m - cjmul(u[3 * b + k], AB[3 * a + k]);  // -(B U^+)_{ab}
      }
      M[3 * a + b] = m;
    }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void force_kernel(Geom g, Links<double> L, Field<double> X, Field<double> Y,
                                                    int n_rhs, double kappa, d2* out, int n_slices) {
  extern __shared__ __align__(16) unsigned char force_lds[];
  cpx<double>(*part)[64][9] = reinterpret_cast<cpx<double>(*)[64][9]>(force_lds);  // [y][site][9]
  // Workgroup b runs on XCD b % 8.  In each run of 32 workgroups, XCD x gets
  // b = x, x + 8, x + 16, x + 24: the 4 directions of one site block, so the
  // site's own X and Y, which all four read, meet in that XCD's L2.
  const int b = blockIdx.x;
  const int mu = (b >> 3) & 3;
  // lanes walk the half-lattice sites of one parity (coalesced spinor loads)
  const int q = ((b >> 5) * 8 + (b & 7)) * 64 + threadIdx.x;
  const bool valid = q < 2 * g.vh;
  const int par = valid && q >= g.vh ? 1 : 0;
  const int s = valid ? q - par * g.vh : 0;
  const Coords c = site_coords(g, s, par);
  const int t = c.t;
  cpx<double> M[9];
  bool ok = false;
  double sgn = 1.0;
  const int half = threadIdx.y & 1, rstep = blockDim.y >> 1;
  const int r0 = valid ? (int)(threadIdx.y >> 1) : n_rhs;
  switch (mu) {
    case 0: force_partial<0>(g, L, X, Y, half, r0, n_rhs, rstep, par, s, c, ok, sgn, M); break;
    case 1: force_partial<1>(g, L, X, Y, half, r0, n_rhs, rstep, par, s, c, ok, sgn, M); break;
    case 2: force_partial<2>(g, L, X, Y, half, r0, n_rhs, rstep, par, s, c, ok, sgn, M); break;
    default: force_partial<3>(g, L, X, Y, half, r0, n_rhs, rstep, par, s, c, ok, sgn, M); break;
  }
  if (threadIdx.y > 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) part[threadIdx.y][threadIdx.x][k] = M[k];
  }
  __syncthreads();
  if (threadIdx.y != 0 || !valid) return;
  for (int j = 1; j < (int)blockDim.y; ++j)
#pragma unroll
    for (int k = 0; k < 9; ++k) M[k] = M[k] + part[j][threadIdx.x][k];
  cpx<double> G[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) G[k] = {0.0, 0.0};
  if (ok) {
    // H = (M - M^+) / (2i): H_ab = (M_ab - conj(M_ba)) / (2i), traceless part
    cpx<double> H[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        const cpx<double> d = {M[3 * a + b].re - M[3 * b + a].re, M[3 * a + b].im + M[3 * b + a].im};
        H[3 * a + b] = {0.5 * sgn * d.im, -0.5 * sgn * d.re};
      }
    const double tr3 = (H[0].re + H[4].re + H[8].re) / 3.0;
    H[0].re -= tr3;
    H[4].re -= tr3;
    H[8].re -= tr3;
#pragma unroll
    for (int k = 0; k < 9; ++k) G[k] = (-kappa) * H[k];
  }
  const long n_slice_sites = (long)g.lx * g.ly * g.lz;
  d2* dst = out + (((long)mu * n_slices + (t + g.t0)) * n_slice_sites + c.x + (long)g.lx * (c.y + (long)g.ly * c.z)) * 9;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    d2 v;
    v.x = G[k].re;
    v.y = G[k].im;
    dst[k] = v;
  }
}

hipError_t launch_force(const Geom& g, Links<double> links, Field<double> X, Field<double> Y, int n_rhs,
                        double kappa, double* force_canon, int n_link_slices, hipStream_t st) {
  const int nr = n_rhs < 1 ? 1 : (n_rhs < 4 ? n_rhs : 4);  // RHS groups; 2 halves each
  const int site_blocks = (2 * g.vh + 63) / 64;
  const dim3 grid(32 * ((site_blocks + 7) / 8)), block(64, 2 * nr);
  const size_t lds = (size_t)2 * nr * 64 * 9 * sizeof(cpx<double>);
  hipLaunchKernelGGL(force_kernel, grid, block, lds, st, g, links, X, Y, n_rhs, kappa, (d2*)force_canon,
                     n_link_slices);
  return hipGetLastError();
}

}  // namespace mfq
