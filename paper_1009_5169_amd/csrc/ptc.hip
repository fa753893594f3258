// Gauge-covariant parallel-transport convolution (PTC) network: the learned
// preconditioner of the flexible GMRES solve.
//
// Paths p = 0..8: p = 0 the identity, p = 1 + mu the forward transport
// (T_p psi)(n) = U_mu(n) psi(n + mu), p = 5 + mu the backward transport
// (T_p psi)(n) = U_mu(n - mu)^+ psi(n - mu), with the Wilson operator's time
// boundary rules.  A layer maps channels c -> c':
//     psi'[c'](n) = sum_c sum_p W[p][c'][c] (T_p psi[c])(n),
// W a complex 4x4 spin matrix.  The network is 1 -> 8 -> 1 channels, linear.
// Layer 1 transports then mixes; layer 2 mixes then transports (W acts on
// spin, T on colour, so they commute), which needs 8 transports per site
// instead of 64.  The forward, backward (adjoint and weight gradient) and
// Adam kernels here are what the library trains the network with.
//
// Channel fields are FP32 Field<float> with virtual RHS index r * C + c.
#include "internal.h"
#include "hop_impl.h"
#include "ptc.h"

namespace mfq {

// Transport along path p (1..8) from the neighbour of (c) to site n: returns
// false across an SF boundary.  nb_site/nb_par give the neighbour; the caller
// loads the neighbour spinor and applies U or U^+.
struct PathHop {
  int site;      // neighbour half-lattice index (parity 1 - par)
  int link_par;  // parity of the site that holds the link
  int link_site;
  float sgn;
  bool ok;
};

__device__ __forceinline__ PathHop path_hop(const Geom& g, const Coords& c, int s, int par, int mu, bool fwd) {
  PathHop h;
  int x = c.x, y = c.y, z = c.z, t = c.t;
  h.sgn = 1.f;
  h.ok = true;
  const int d = fwd ? 1 : -1;
  if (mu == 0) {
    t += d;
    if (t == g.td || t < 0) {
      if (g.bc == BC_SF) h.ok = false;
      t = t < 0 ? g.td - 1 : 0;
      if (g.bc == BC_ANTIPERIODIC) h.sgn = -1.f;
    }
  } else if (mu == 1) {
    x = (x + d + g.lx) % g.lx;
  } else if (mu == 2) {
    y = (y + d + g.ly) % g.ly;
  } else {
    z = (z + d + g.lz) % g.lz;
  }
  h.site = half_index(g, x, y, z, t);
  h.link_par = fwd ? par : 1 - par;
  h.link_site = fwd ? s : h.site;
  return h;
}

// out = U psi (fwd) or U^+ psi (bwd), scaled by sgn
template <typename T>
__device__ __forceinline__ void colour_mul(const cpx<T> u[9], bool dag, T sgn, const Spinor<T>& in, Spinor<T>& out) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<T> acc = {(T)0, (T)0};
#pragma unroll
      for (int b = 0; b < 3; ++b)
        acc = acc + (dag ? cjmul(u[3 * b + a], in.v[3 * sp + b]) : cmul(u[3 * a + b], in.v[3 * sp + b]));
      out.v[3 * sp + a] = sgn * acc;
    }
}

// acc += W psi on spin (W: 16 complex, row-major [s'][s])
__device__ __forceinline__ void spin_mul_add(const f2* W, const Spinor<float>& in, Spinor<float>& acc) {
#pragma unroll
  for (int so = 0; so < 4; ++so)
#pragma unroll
    for (int si = 0; si < 4; ++si) {
      const f2 w = W[4 * so + si];
      const cpx<float> wc = {w.x, w.y};
#pragma unroll
      for (int a = 0; a < 3; ++a) acc.v[3 * so + a] = acc.v[3 * so + a] + cmul(wc, in.v[3 * si + a]);
    }
}

// acc += W^+ psi on spin
__device__ __forceinline__ void spin_mul_add_dag(const f2* W, const Spinor<float>& in, Spinor<float>& acc) {
#pragma unroll
  for (int so = 0; so < 4; ++so)
#pragma unroll
    for (int si = 0; si < 4; ++si) {
      const f2 w = W[4 * si + so];  // (W^+)_{so,si} = conj(W_{si,so})
      const cpx<float> wc = {w.x, w.y};
#pragma unroll
      for (int a = 0; a < 3; ++a) acc.v[3 * so + a] = acc.v[3 * so + a] + cjmul(wc, in.v[3 * si + a]);
    }
}

template <typename T>
__device__ __forceinline__ void zero_sp(Spinor<T>& a) {
#pragma unroll
  for (int k = 0; k < 12; ++k) a.v[k] = {(T)0, (T)0};
}

// T_p psi at site (s, par) for field f, virtual RHS index vr
template <typename SI>
__device__ __forceinline__ void transported(const Geom& g, const Links<float>& L, const Field<SI>& f, int vr, int p,
                                            int s, int par, const Coords& c, Spinor<float>& out) {
  if (p == 0) {
    load_spinor(f, vr, par, s, out);
    return;
  }
  const int mu = p <= 4 ? p - 1 : p - 5;
  const bool fwd = p <= 4;
  const PathHop h = path_hop(g, c, s, par, mu, fwd);
  if (!h.ok) {
    zero_sp(out);
    return;
  }
  Spinor<float> nb;
  load_spinor(f, vr, 1 - par, h.site, nb);
  cpx<float> u[9];
  load_link(L, h.link_par, mu, h.link_site, u);
  colour_mul(u, !fwd, h.sgn, nb, out);
}

#define PTC_LANE                                                   \
  const int q = blockIdx.x * blockDim.x + threadIdx.x;             \
  const int r = blockIdx.y;                                        \
  if (q >= 2 * g.vh || r >= n_rhs) return;                         \
  const int par = q >= g.vh ? 1 : 0;                               \
  const int s = q - par * g.vh;                                    \
  const Coords c = site_coords(g, s, par);

// Layer 1 (1 -> 8): hid[r*8 + c'] = sum_p W1[p][c'] (T_p in_r); grid.z picks
// a group of 4 output channels.
template <typename SI>
__global__ __launch_bounds__(256) void ptc_l1_kernel(Geom g, Links<float> L, Field<SI> in, Field<float> hid,
                                                     const f2* W1, int n_rhs, float scale) {
  PTC_LANE
  const int c0 = blockIdx.z * 4;
  Spinor<float> acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) zero_sp(acc[k]);
  for (int p = 0; p < PTC_PATHS; ++p) {
    Spinor<float> t;
    transported(g, L, in, r, p, s, par, c, t);
#pragma unroll
    for (int k = 0; k < 4; ++k) spin_mul_add(W1 + (p * PTC_HIDDEN + c0 + k) * 16, t, acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int j = 0; j < 12; ++j) acc[k].v[j] = scale * acc[k].v[j];
    store_spinor(hid, r * PTC_HIDDEN + c0 + k, par, s, acc[k]);
  }
}

// Layer 2 (8 -> 1): out_r = sum_p T_p chi_p, chi_p = sum_c W2[p][c] hid[r*8+c].
template <typename SO>
__global__ __launch_bounds__(256) void ptc_l2_kernel(Geom g, Links<float> L, Field<float> hid, Field<SO> out,
                                                     const f2* W2, int n_rhs, float scale) {
  PTC_LANE
  Spinor<float> acc;
  zero_sp(acc);
  for (int p = 0; p < PTC_PATHS; ++p) {
    int ms = s, mpar = par;
    PathHop h;
    int mu = 0;
    bool fwd = true;
    if (p > 0) {
      mu = p <= 4 ? p - 1 : p - 5;
      fwd = p <= 4;
      h = path_hop(g, c, s, par, mu, fwd);
      if (!h.ok) continue;
      ms = h.site;
      mpar = 1 - par;
    }
    Spinor<float> chi;
    zero_sp(chi);
    for (int k = 0; k < PTC_HIDDEN; ++k) {
      Spinor<float> x;
      load_spinor(hid, r * PTC_HIDDEN + k, mpar, ms, x);
      spin_mul_add(W2 + (p * PTC_HIDDEN + k) * 16, x, chi);
    }
    if (p == 0) {
#pragma unroll
      for (int j = 0; j < 12; ++j) acc.v[j] = acc.v[j] + chi.v[j];
    } else {
      cpx<float> u[9];
      load_link(L, h.link_par, mu, h.link_site, u);
      Spinor<float> t;
      colour_mul(u, !fwd, h.sgn, chi, t);
#pragma unroll
      for (int j = 0; j < 12; ++j) acc.v[j] = acc.v[j] + t.v[j];
    }
  }
#pragma unroll
  for (int j = 0; j < 12; ++j) acc.v[j] = scale * acc.v[j];
  store_spinor(out, r, par, s, acc);
}

template <typename SI, typename SO>
hipError_t ptc_forward(const Geom& g, Links<float> L, Field<SI> in, Field<float> hid, Field<SO> out, const f2* W1,
                       const f2* W2, int n_rhs, float in_scale, float out_scale, hipStream_t st) {
  const dim3 grid1((2 * g.vh + 255) / 256, n_rhs, PTC_HIDDEN / 4);
  hipLaunchKernelGGL((ptc_l1_kernel<SI>), grid1, dim3(256), 0, st, g, L, in, hid, W1, n_rhs, in_scale);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 grid2((2 * g.vh + 255) / 256, n_rhs);
  hipLaunchKernelGGL((ptc_l2_kernel<SO>), grid2, dim3(256), 0, st, g, L, hid, out, W2, n_rhs, out_scale);
  return hipGetLastError();
}

template hipError_t ptc_forward<double, double>(const Geom&, Links<float>, Field<double>, Field<float>, Field<double>,
                                                const f2*, const f2*, int, float, float, hipStream_t);
template hipError_t ptc_forward<double, float>(const Geom&, Links<float>, Field<double>, Field<float>, Field<float>,
                                               const f2*, const f2*, int, float, float, hipStream_t);
template hipError_t ptc_forward<float, float>(const Geom&, Links<float>, Field<float>, Field<float>, Field<float>,
                                              const f2*, const f2*, int, float, float, hipStream_t);

}  // namespace mfq

namespace mfq {

// ---------------------------------------------------------------- backward
// Adjoint of layer 2 in its input.  T_p^+ = T_pbar (the forward transport's
// adjoint is the backward one), and W commutes with transports, so
//   gh[c](n) = sum_p W2[p][c]^+ (T_pbar gy)(n).
__global__ __launch_bounds__(256) void ptc_adj2_kernel(Geom g, Links<float> L, Field<float> gy, Field<float> gh,
                                                       const f2* W2, int n_rhs) {
  PTC_LANE
  const int c0 = blockIdx.z * 4;
  Spinor<float> acc[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) zero_sp(acc[k]);
  for (int p = 0; p < PTC_PATHS; ++p) {
    const int pbar = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
    Spinor<float> t;
    transported(g, L, gy, r, pbar, s, par, c, t);
#pragma unroll
    for (int k = 0; k < 4; ++k) spin_mul_add_dag(W2 + (p * PTC_HIDDEN + c0 + k) * 16, t, acc[k]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) store_spinor(gh, r * PTC_HIDDEN + c0 + k, par, s, acc[k]);
}

hipError_t ptc_adjoint2(const Geom& g, Links<float> L, Field<float> gy, Field<float> gh, const f2* W2, int n_pairs,
                        hipStream_t st) {
  const dim3 grid((2 * g.vh + 255) / 256, n_pairs, PTC_HIDDEN / 4);
  hipLaunchKernelGGL(ptc_adj2_kernel, grid, dim3(256), 0, st, g, L, gy, gh, W2, n_pairs);
  return hipGetLastError();
}

// Weight gradients: blockIdx.y = (path, c_in) and blockIdx.z a group of CO
// output channels; each thread transports its site's input once per pair and
// sums the spin outer products with the CO output gradients over colours and
// pairs; the workgroup reduces in FP64 and writes one partial per (path,
// c_out, c_in) block and workgroup.
template <typename SX, int CO>
__global__ __launch_bounds__(256) void ptc_wgrad_kernel(Geom g, Links<float> L, Field<SX> x, int c_in, Field<float> gf,
                                                        int c_out, int n_pairs, double* part) {
  __shared__ double ws[4][CO * 32];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int ci = blockIdx.y % c_in;
  const int p = blockIdx.y / c_in;
  const int co0 = blockIdx.z * CO;
  float acc[CO][32];
#pragma unroll
  for (int j = 0; j < CO; ++j)
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[j][k] = 0.f;
  if (q < 2 * g.vh) {
    const int par = q >= g.vh ? 1 : 0;
    const int s = q - par * g.vh;
    const Coords c = site_coords(g, s, par);
    for (int k = 0; k < n_pairs; ++k) {
      Spinor<float> t;
      transported(g, L, x, k * c_in + ci, p, s, par, c, t);
#pragma unroll
      for (int j = 0; j < CO; ++j) {
        Spinor<float> gg;
        load_spinor(gf, k * c_out + co0 + j, par, s, gg);
#pragma unroll
        for (int so = 0; so < 4; ++so)
#pragma unroll
          for (int si = 0; si < 4; ++si) {
            cpx<float> o = {0.f, 0.f};
#pragma unroll
            for (int a = 0; a < 3; ++a) o = o + cjmul(t.v[3 * si + a], gg.v[3 * so + a]);
            acc[j][2 * (4 * so + si)] += o.re;
            acc[j][2 * (4 * so + si) + 1] += o.im;
          }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < CO; ++j)
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const double v = wave_sum((double)acc[j][k]);
      if (lane == 0) ws[wave][j * 32 + k] = v;
    }
  __syncthreads();
  if (threadIdx.x < CO * 32) {
    const int j = threadIdx.x / 32, k = threadIdx.x % 32;
    const double v = ((ws[0][threadIdx.x] + ws[1][threadIdx.x]) + ws[2][threadIdx.x]) + ws[3][threadIdx.x];
    const int idx = (p * c_out + co0 + j) * c_in + ci;
    part[((long)idx * gridDim.x + blockIdx.x) * 32 + k] = v;
  }
}

// The same weight gradient with the transport moved onto the output
// gradient: T_p^+ = T_pbar, so
//   sum_n g(n) (T_p x)(n)^+ = sum_m (T_pbar g)(m) x(m)^+,
// and a single-channel g (layer 2: c_out = 1) is transported once per path
// instead of each of the c_in input channels.  blockIdx.y = path, blockIdx.z
// a group of CI input channels; same partial layout as ptc_wgrad_kernel.
template <typename SX, int CI>
__global__ __launch_bounds__(256) void ptc_wgrad_adj_kernel(Geom g, Links<float> L, Field<SX> x, int c_in,
                                                            Field<float> gf, int n_pairs, double* part) {
  __shared__ double ws[4][CI * 32];
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;
  const int pbar = p == 0 ? 0 : (p <= 4 ? p + 4 : p - 4);
  const int ci0 = blockIdx.z * CI;
  float acc[CI][32];
#pragma unroll
  for (int j = 0; j < CI; ++j)
#pragma unroll
    for (int k = 0; k < 32; ++k) acc[j][k] = 0.f;
  if (q < 2 * g.vh) {
    const int par = q >= g.vh ? 1 : 0;
    const int s = q - par * g.vh;
    const Coords c = site_coords(g, s, par);
    for (int k = 0; k < n_pairs; ++k) {
      Spinor<float> tg;
      transported(g, L, gf, k, pbar, s, par, c, tg);
#pragma unroll
      for (int j = 0; j < CI; ++j) {
        Spinor<float> xx;
        load_spinor(x, k * c_in + ci0 + j, par, s, xx);
#pragma unroll
        for (int so = 0; so < 4; ++so)
#pragma unroll
          for (int si = 0; si < 4; ++si) {
            cpx<float> o = {0.f, 0.f};
#pragma unroll
            for (int a = 0; a < 3; ++a) o = o + cjmul(xx.v[3 * si + a], tg.v[3 * so + a]);
            acc[j][2 * (4 * so + si)] += o.re;
            acc[j][2 * (4 * so + si) + 1] += o.im;
          }
      }
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < CI; ++j)
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      const double v = wave_sum((double)acc[j][k]);
      if (lane == 0) ws[wave][j * 32 + k] = v;
    }
  __syncthreads();
  if (threadIdx.x < CI * 32) {
    const int j = threadIdx.x / 32, k = threadIdx.x % 32;
    const double v = ((ws[0][threadIdx.x] + ws[1][threadIdx.x]) + ws[2][threadIdx.x]) + ws[3][threadIdx.x];
    const int idx = p * c_in + ci0 + j;  // (p * c_out + co) * c_in + ci with c_out = 1
    part[((long)idx * gridDim.x + blockIdx.x) * 32 + k] = v;
  }
}

__global__ void ptc_grad_reduce_kernel(const double* part, int nblk, int n_idx, double* grad) {
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;  // one wave per (idx, component)
  const int lane = threadIdx.x & 63;
  if (w >= n_idx * 32) return;
  const int idx = w / 32, k = w % 32;
  double v = 0.0;
  for (int j = lane; j < nblk; j += 64) v += part[((long)idx * nblk + j) * 32 + k];
  v = wave_sum(v);
  if (lane == 0) grad[(long)idx * 32 + k] = v;
}

template <typename SX>
hipError_t ptc_weight_grad(const Geom& g, Links<float> L, Field<SX> x, int c_in, Field<float> gf, int c_out,
                           int n_pairs, double* part, double* grad, hipStream_t st) {
  const int nblk = (2 * g.vh + 255) / 256;
  const int n_idx = PTC_PATHS * c_in * c_out;
  if (c_out == 1 && c_in % 4 == 0)
    hipLaunchKernelGGL((ptc_wgrad_adj_kernel<SX, 4>), dim3(nblk, PTC_PATHS, c_in / 4), dim3(256), 0, st, g, L, x,
                       c_in, gf, n_pairs, part);
  else if (c_out % 4 == 0)
    hipLaunchKernelGGL((ptc_wgrad_kernel<SX, 4>), dim3(nblk, PTC_PATHS * c_in, c_out / 4), dim3(256), 0, st, g, L, x,
                       c_in, gf, c_out, n_pairs, part);
  else
    hipLaunchKernelGGL((ptc_wgrad_kernel<SX, 1>), dim3(nblk, PTC_PATHS * c_in, c_out), dim3(256), 0, st, g, L, x,
                       c_in, gf, c_out, n_pairs, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int waves = n_idx * 32;
  hipLaunchKernelGGL(ptc_grad_reduce_kernel, dim3((waves + 3) / 4), dim3(256), 0, st, part, nblk, n_idx, grad);
  return hipGetLastError();
}

template hipError_t ptc_weight_grad<double>(const Geom&, Links<float>, Field<double>, int, Field<float>, int, int,
                                            double*, double*, hipStream_t);
template hipError_t ptc_weight_grad<float>(const Geom&, Links<float>, Field<float>, int, Field<float>, int, int,
                                           double*, double*, hipStream_t);

__global__ __launch_bounds__(256) void ptc_loss_kernel(Geom g, Field<float> y, Field<double> e, const double* enorm2,
                                                       Field<float> gy, int n_rhs, double* part) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = blockIdx.y;
  double red = 0.0;
  if (q < 2 * g.vh) {
    const int par = q >= g.vh ? 1 : 0;
    const int s = q - par * g.vh;
    Spinor<float> yy;
    Spinor<double> ee;
    load_spinor(y, r, par, s, yy);
    load_spinor(e, r, par, s, ee);
    const double en = enorm2[r] > 0.0 ? enorm2[r] : 1.0;  // a zero error contributes |y|^2
    const float sc = (float)(2.0 / (n_rhs * en));
    Spinor<float> d;
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      const double dr = (double)yy.v[k].re - ee.v[k].re, di = (double)yy.v[k].im - ee.v[k].im;
      red += dr * dr + di * di;
      d.v[k] = {sc * (float)dr, sc * (float)di};
    }
    red /= en;
    store_spinor(gy, r, par, s, d);
  }
  red = wave_sum(red);
  __shared__ double ws[4];
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = red;
  __syncthreads();
  if (threadIdx.x == 0) part[(long)r * gridDim.x + blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

hipError_t ptc_loss_grad_out(const Geom& g, Field<float> y, Field<double> e, const double* enorm2, Field<float> gy,
                             int n_pairs, double* part, hipStream_t st) {
  hipLaunchKernelGGL(ptc_loss_kernel, dim3((2 * g.vh + 255) / 256, n_pairs), dim3(256), 0, st, g, y, e, enorm2, gy,
                     n_pairs, part);
  return hipGetLastError();
}

// Round to the nearest BF16 value (ties to even), kept in an FP32 register.
__device__ __forceinline__ float round_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// One Adam step (Kingma and Ba, Algorithm 1) on FP32 master weights, Re and Im
// separate parameters.  The coefficients that depend only on beta and t
// (1 - beta, 1 - beta^t) come from the host in FP64 and are rounded once:
// forming 1 - beta in FP32 from beta = 0.999f would be off by 1.3e-5.
__global__ void ptc_adam_kernel(float* w, const double* grad, float* m, float* v, int n_real, float lr, float b1,
                                float c1, float b2, float c2, float inv_bc1, float inv_bc2, float eps,
                                float* w_infer) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_real) return;
  const float gr = (float)grad[i];
  const float mi = b1 * m[i] + c1 * gr;
  const float vi = b2 * v[i] + c2 * (gr * gr);
  m[i] = mi;
  v[i] = vi;
  const float mh = mi * inv_bc1;
  const float vh = vi * inv_bc2;
  const float wi = w[i] - lr * mh / (sqrtf(vh) + eps);
  w[i] = wi;
  w_infer[i] = round_bf16(wi);
}

hipError_t ptc_adam(float* w, const double* grad, float* m, float* v, int n_real, int t, double lr, double b1,
                    double b2, double eps, f2* w_infer, hipStream_t st) {
  const double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
  hipLaunchKernelGGL(ptc_adam_kernel, dim3((n_real + 255) / 256), dim3(256), 0, st, w, grad, m, v, n_real, (float)lr,
                     (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)(1.0 / bc1),
                     (float)(1.0 / bc2), (float)eps, (float*)w_infer);
  return hipGetLastError();
}

}  // namespace mfq

namespace mfq {

// ------------------------------------------------- matrix-core forward pass
// Both channel mixings are complex matrix products over (channel, spin) that
// leave colour alone, so for each colour they are real matrix products over
// sites once a complex weight w = wr + i wi is written as the 2x2 real block
// [[wr, -wi], [wi, wr]] acting on (re, im).  They run on the 16x16x32 BF16
// matrix instruction in transposed form: rows are output components, the 16
// columns are 16 sites of one parity and one right-hand side, so each lane's
// results belong to one site and stores coalesce across lanes.
//
//   layer 1:  K = 9 paths x 4 spins x (re, im) = 72, padded to 96 (3 steps),
//             M = 8 channels x 4 spins x (re, im) = 64 (4 tiles);
//   layer 2:  chi_p = sum_c W2[p][c] h_c is formed at the site that holds h
//             (the mixing acts on spin, the transport on colour, so they
//             commute): K = 64 hidden components taken straight from layer
//             1's accumulators (2 steps), M = 9 paths x 4 spins x (re, im) =
//             72, padded to 80 (5 tiles).
// The chi_p go to memory (FP32) and a gather kernel forms
// out(n) = chi_0(n) + sum_{p>0} (T_p chi_p)(n); the hidden field never leaves
// registers.
//
// Weights are BF16 values (the inference copy) and so exact as BF16
// operands.  Each FP32 activation x is split as hi = bf16(x),
// lo = bf16(x - hi), |x - hi - lo| <= 2^-18 |x|, and both halves go through
// the matrix unit with FP32 accumulation, so the products are those of FP32
// activations to that relative accuracy.
//
// Operand layouts of the instruction (lane l, group g = l / 16, element i of
// the 8-vector): A: row l % 16, k = 8 g + i;  B: column l % 16, k = 8 g + i;
// result element e: column l % 16, row 4 g + e.
//
// Layer 1's k order lets the four lane groups of a site transport the same
// paths: in step j, group g holds k = 32 j + 8 g + 2 q + ri for path
// p = 4 j + q and spin g, so each lane transports one spin of four paths.
// Layer 2's k order is the order in which layer 1's result elements sit in
// the lanes: step j, group g, element i is hidden row
// 16 (2 j + i / 4) + 4 g + (i % 4).

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int MX_L1_TILES = 4, MX_L1_STEPS = 3, MX_L2_TILES = 5, MX_L2_STEPS = 2;
constexpr int MX_L1_OPS = MX_L1_TILES * MX_L1_STEPS;
constexpr int MX_OPS = (MX_L1_OPS + MX_L2_TILES * MX_L2_STEPS) * 64;  // 16-byte operands, lane-major
constexpr int MX_CHI = PTC_PATHS * 2 * 24;  // floats per (rhs, site pair) of chi: [p][parity][24]

// entry of the real 2x2 block of w at (output re/im ro, input re/im ri)
__device__ __forceinline__ float re_block(f2 w, int ro, int ri) { return ro == ri ? w.x : (ro == 0 ? -w.y : w.y); }

__global__ void ptc_pack_ops_kernel(const f2* W1, const f2* W2, f4* ops_out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= MX_OPS) return;
  const int l = idx % 64, o = idx / 64, row = l % 16, grp = l / 16;
  bf16x8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    float x = 0.f;
    if (o < MX_L1_OPS) {
      const int t = o / MX_L1_STEPS, j = o % MX_L1_STEPS;
      const int n = 16 * t + row;  // hidden component: channel n/8, spin (n%8)/2, re/im n%2
      const int p = 4 * j + i / 2, si = grp, ri = i % 2;
      if (p < PTC_PATHS) x = re_block(W1[(p * PTC_HIDDEN + n / 8) * 16 + ((n % 8) / 2) * 4 + si], n % 2, ri);
    } else {
      const int o2 = o - MX_L1_OPS;
      const int t = o2 / MX_L2_STEPS, j = o2 % MX_L2_STEPS;
      const int m = 16 * t + row;                                // chi component: path m/8, spin (m%8)/2, re/im m%2
      const int n = 16 * (2 * j + i / 4) + 4 * grp + (i % 4);  // hidden component fed at this k
      if (m < PTC_PATHS * 8)
        x = re_block(W2[((m / 8) * PTC_HIDDEN + n / 8) * 16 + ((m % 8) / 2) * 4 + (n % 8) / 2], m % 2, n % 2);
    }
    v[i] = (__bf16)x;
  }
  __builtin_memcpy(&ops_out[idx], &v, sizeof(v));
}

hipError_t ptc_pack_ops(const f2* W1, const f2* W2, void* ops, hipStream_t st) {
  hipLaunchKernelGGL(ptc_pack_ops_kernel, dim3((MX_OPS + 255) / 256), dim3(256), 0, st, W1, W2, (f4*)ops);
  return hipGetLastError();
}

size_t ptc_ops_bytes() { return (size_t)MX_OPS * 16; }
size_t ptc_chi_floats(const Geom& g, int n_rhs) { return (size_t)n_rhs * MX_CHI * g.vs; }

// spin sp of a spinor: v[a]
__device__ __forceinline__ void load_spin(const Field<double>& f, int vr, int par, int s, int sp, cpx<float> v[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const d2 q = f.data[f.cidx(vr, par, 3 * sp + a, s)];
    v[a] = {(float)q.x, (float)q.y};
  }
}

// (T_P psi)(s) restricted to spin sp; zero across an SF boundary and for
// lanes past the end of the half lattice.
template <int P, typename SI>
__device__ __forceinline__ void spin_transport(const Geom& g, const Links<float>& L, const Field<SI>& f, int vr, int s,
                                               int par, const Coords& c, int sp, bool valid, cpx<float> y[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) y[k] = {0.f, 0.f};
  if constexpr (P >= PTC_PATHS) {
    return;
  } else if constexpr (P == 0) {
    if (valid) load_spin(f, vr, par, s, sp, y);
  } else {
    constexpr int mu = P <= 4 ? P - 1 : P - 5;
    constexpr bool fwd = P <= 4;
    const PathHop ph = path_hop(g, c, s, par, mu, fwd);
    if (!valid || !ph.ok) return;
    cpx<float> x[3], u[9];
    load_spin(f, vr, 1 - par, ph.site, sp, x);
    load_link(L, ph.link_par, mu, ph.link_site, u);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<float> acc = {0.f, 0.f};
#pragma unroll
      for (int b = 0; b < 3; ++b) acc = acc + (fwd ? cmul(u[3 * a + b], x[b]) : cjmul(u[3 * b + a], x[b]));
      y[a] = ph.sgn * acc;
    }
  }
}

__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = (__bf16)x;
  lo = (__bf16)(x - (float)hi);
}

#define MX_MFMA(a, b, c) __builtin_amdgcn_mfma_f32_16x16x32_bf16((a), (b), (c), 0, 0, 0)
#define MX_SCHED_FENCE __builtin_amdgcn_sched_barrier(0);

// One layer-1 K step: paths 4J .. 4J+3, spin g, 4 tiles, 3 colours.
template <int J, typename SI>
__device__ __forceinline__ void mx_l1_step(const Geom& g, const Links<float>& L, const Field<SI>& in, int r, int s,
                                           int par, const Coords& c, int grp, bool valid,
                                           const bf16x8* wops, int lane, floatx4 (&acc)[3][MX_L1_TILES]) {
  cpx<float> y[4][3];
  spin_transport<4 * J + 0>(g, L, in, r, s, par, c, grp, valid, y[0]);
  spin_transport<4 * J + 1>(g, L, in, r, s, par, c, grp, valid, y[1]);
  spin_transport<4 * J + 2>(g, L, in, r, s, par, c, grp, valid, y[2]);
  spin_transport<4 * J + 3>(g, L, in, r, s, par, c, grp, valid, y[3]);
  bf16x8 bh[3], bl[3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      __bf16 hi, lo;
      split_bf16(y[q][a].re, hi, lo);
      bh[a][2 * q] = hi;
      bl[a][2 * q] = lo;
      split_bf16(y[q][a].im, hi, lo);
      bh[a][2 * q + 1] = hi;
      bl[a][2 * q + 1] = lo;
    }
#pragma unroll
  for (int t = 0; t < MX_L1_TILES; ++t) {
    const bf16x8 w = wops[(t * MX_L1_STEPS + J) * 64 + lane];
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a][t] = MX_MFMA(w, bh[a], acc[a][t]);
#pragma unroll
    for (int a = 0; a < 3; ++a) acc[a][t] = MX_MFMA(w, bl[a], acc[a][t]);
  }
}

// One wavefront per 16 sites of one parity and one right-hand side (a tile);
// waves loop over tiles.  The operands of both weight matrices are staged in
// LDS once per workgroup.  Scheduling fences between the K steps keep the
// compiler from hoisting every step's neighbour loads to the top, which
// would take the register count past two waves per SIMD.
template <typename SI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ptc_mx_kernel(Geom g, Links<float> L, Field<SI> in, float* chi, const f4* ops,
                                                     int n_tiles) {
  __shared__ bf16x8 wops[MX_OPS];
  for (int i = threadIdx.x; i < MX_OPS; i += blockDim.x) __builtin_memcpy(&wops[i], &ops[i], 16);
  __syncthreads();
  const int lane = threadIdx.x & 63, grp = lane >> 4;
  const int tpp = (g.vh + 15) / 16;  // tiles per parity
  for (int tile = blockIdx.x * 4 + (threadIdx.x >> 6); tile < n_tiles; tile += gridDim.x * 4) {
    const int r = tile / (2 * tpp);
    const int par = (tile / tpp) & 1;
    const int s0 = (tile % tpp) * 16 + (lane & 15);
    const bool valid = s0 < g.vh;
    const int s = valid ? s0 : 0;
    const Coords c = site_coords(g, s, par);
    floatx4 acc[3][MX_L1_TILES];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int t = 0; t < MX_L1_TILES; ++t) acc[a][t] = floatx4{0.f, 0.f, 0.f, 0.f};
    mx_l1_step<0>(g, L, in, r, s, par, c, grp, valid, wops, lane, acc);
    MX_SCHED_FENCE
    mx_l1_step<1>(g, L, in, r, s, par, c, grp, valid, wops, lane, acc);
    MX_SCHED_FENCE
    mx_l1_step<2>(g, L, in, r, s, par, c, grp, valid, wops, lane, acc);
    MX_SCHED_FENCE
    float* base = chi + ((long)r * MX_CHI + par * 24) * g.vs + s;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      bf16x8 bh[MX_L2_STEPS], bl[MX_L2_STEPS];
#pragma unroll
      for (int j = 0; j < MX_L2_STEPS; ++j)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          __bf16 hi, lo;
          split_bf16(acc[a][2 * j + i / 4][i % 4], hi, lo);
          bh[j][i] = hi;
          bl[j][i] = lo;
        }
      floatx4 o[MX_L2_TILES];
#pragma unroll
      for (int t = 0; t < MX_L2_TILES; ++t) o[t] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < MX_L2_STEPS; ++j)
#pragma unroll
        for (int t = 0; t < MX_L2_TILES; ++t) {
          const bf16x8 w = wops[(MX_L1_OPS + t * MX_L2_STEPS + j) * 64 + lane];
          o[t] = MX_MFMA(w, bh[j], o[t]);
          o[t] = MX_MFMA(w, bl[j], o[t]);
        }
      if (valid) {
        // row 16 t + 4 g + e = (path 2 t + g / 2, spin 2 (g % 2) + e / 2, re/im e % 2)
#pragma unroll
        for (int t = 0; t < MX_L2_TILES; ++t) {
          const int p = 2 * t + grp / 2;
          if (p < PTC_PATHS) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              const int so = 2 * (grp % 2) + e / 2;
              base[((long)p * 48 + (3 * so + a) * 2 + (e % 2)) * g.vs] = o[t][e];
            }
          }
        }
      }
    }
  }
}

// out(n) = chi_0(n) + sum_{p>0} (T_p chi_p)(n); chi is [rhs][p][parity][24][vs].
template <typename SO>
__global__ __launch_bounds__(256) void ptc_gather_kernel(Geom g, Links<float> L, const float* chi, Field<SO> out,
                                                         int n_rhs) {
  PTC_LANE
  const float* cr = chi + (long)r * MX_CHI * g.vs;
  Spinor<float> acc;
#pragma unroll
  for (int k = 0; k < 12; ++k) acc.v[k] = {cr[(par * 24 + 2 * k) * (long)g.vs + s], cr[(par * 24 + 2 * k + 1) * (long)g.vs + s]};
#pragma unroll
  for (int p = 1; p < PTC_PATHS; ++p) {
    const int mu = p <= 4 ? p - 1 : p - 5;
    const bool fwd = p <= 4;
    const PathHop ph = path_hop(g, c, s, par, mu, fwd);
    if (!ph.ok) continue;
    const float* cp = cr + ((long)p * 48 + (1 - par) * 24) * g.vs + ph.site;
    Spinor<float> x, t;
#pragma unroll
    for (int k = 0; k < 12; ++k) x.v[k] = {cp[(2 * k) * (long)g.vs], cp[(2 * k + 1) * (long)g.vs]};
    cpx<float> u[9];
    load_link(L, ph.link_par, mu, ph.link_site, u);
    colour_mul(u, !fwd, ph.sgn, x, t);
#pragma unroll
    for (int k = 0; k < 12; ++k) acc.v[k] = acc.v[k] + t.v[k];
  }
  store_spinor(out, r, par, s, acc);
}

template <typename SI, typename SO>
hipError_t ptc_forward_mx(const Geom& g, Links<float> L, Field<SI> in, float* chi, Field<SO> out, const void* ops,
                          int n_rhs, hipStream_t st) {
  const int n_tiles = n_rhs * 2 * ((g.vh + 15) / 16);
  int blocks = (n_tiles + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((ptc_mx_kernel<SI>), dim3(blocks), dim3(256), 0, st, g, L, in, chi, (const f4*)ops, n_tiles);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((ptc_gather_kernel<SO>), dim3((2 * g.vh + 255) / 256, n_rhs), dim3(256), 0, st, g, L, chi, out,
                     n_rhs);
  return hipGetLastError();
}

template hipError_t ptc_forward_mx<double, double>(const Geom&, Links<float>, Field<double>, float*, Field<double>,
                                                   const void*, int, hipStream_t);

}  // namespace mfq
