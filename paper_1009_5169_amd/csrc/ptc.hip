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
// instead of 64.  Inference, the training forward pass, the adjoint of
// layer 2 and both weight gradients run on the BF16 matrix instruction (FP32
// values split into hi and lo halves); Adam updates FP32 master weights.
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

#define PTC_LANE                                                   \
  const int q = blockIdx.x * blockDim.x + threadIdx.x;             \
  const int r = blockIdx.y;                                        \
  if (q >= 2 * g.vh || r >= n_rhs) return;                         \
  const int par = q >= g.vh ? 1 : 0;                               \
  const int s = q - par * g.vh;                                    \
  const Coords c = site_coords(g, s, par);

}  // namespace mfq

namespace mfq {

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

// part 0: the weights as BF16 (the inference copy is BF16-valued, so exact);
// part 1 / 2: the hi / lo halves of FP32 weights (hi = bf16(w), lo = bf16(w - hi)).
__global__ void ptc_pack_ops_kernel(const f2* W1, const f2* W2, f4* ops_out, int part) {
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
    const __bf16 hi = (__bf16)x;
    v[i] = part == 2 ? (__bf16)(x - (float)hi) : hi;
  }
  __builtin_memcpy(&ops_out[idx], &v, sizeof(v));
}

hipError_t ptc_pack_ops(const f2* W1, const f2* W2, void* ops, hipStream_t st) {
  hipLaunchKernelGGL(ptc_pack_ops_kernel, dim3((MX_OPS + 255) / 256), dim3(256), 0, st, W1, W2, (f4*)ops, 0);
  return hipGetLastError();
}

hipError_t ptc_pack_ops_split(const f2* W1, const f2* W2, void* ops, hipStream_t st) {
  hipLaunchKernelGGL(ptc_pack_ops_kernel, dim3((MX_OPS + 255) / 256), dim3(256), 0, st, W1, W2, (f4*)ops, 1);
  hipLaunchKernelGGL(ptc_pack_ops_kernel, dim3((MX_OPS + 255) / 256), dim3(256), 0, st, W1, W2, (f4*)ops + MX_OPS, 2);
  return hipGetLastError();
}

// Wa[q][c] = W2[qbar][c]^+ (spin adjoint): the adjoint of layer 2 is then a
// layer-1 map, gh[c] = sum_q Wa[q][c] (T_q gy).
__global__ void ptc_adj_weights_kernel(const f2* W2, f2* Wa) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= PTC_W1) return;
  const int e = i % 16, qc = i / 16, c = qc % PTC_HIDDEN, q = qc / PTC_HIDDEN;
  const int so = e / 4, si = e % 4;
  const int p = q == 0 ? 0 : (q <= 4 ? q + 4 : q - 4);
  const f2 w = W2[(p * PTC_HIDDEN + c) * 16 + si * 4 + so];
  Wa[i] = f2{w.x, -w.y};
}

hipError_t ptc_adj_weights(const f2* W2, f2* Wa, hipStream_t st) {
  hipLaunchKernelGGL(ptc_adj_weights_kernel, dim3((PTC_W1 + 255) / 256), dim3(256), 0, st, W2, Wa);
  return hipGetLastError();
}

size_t ptc_ops_bytes() { return (size_t)MX_OPS * 16; }
size_t ptc_chi_floats(const Geom& g, int n_rhs) { return (size_t)n_rhs * MX_CHI * g.vs; }


// colours of spin sp of the spinor at (vr, par, s)
template <typename SF>
__device__ __forceinline__ void load_spin_any(const Field<SF>& f, int vr, int par, int s, int sp, cpx<float> v[3]) {
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    const int comp = 3 * sp + b;
    if constexpr (sizeof(SF) == 8) {
      const d2 q = f.data[f.cidx(vr, par, comp, s)];
      v[b] = {(float)q.x, (float)q.y};
    } else {
      const f4 q = f.data[f.cidx(vr, par, comp / 2, s)];
      v[b] = (comp & 1) ? cpx<float>{q.z, q.w} : cpx<float>{q.x, q.y};
    }
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
    if (valid) load_spin_any(f, vr, par, s, sp, y);
  } else {
    constexpr int mu = P <= 4 ? P - 1 : P - 5;
    constexpr bool fwd = P <= 4;
    const PathHop ph = path_hop(g, c, s, par, mu, fwd);
    if (!valid || !ph.ok) return;
    cpx<float> x[3], u[9];
    load_spin_any(f, vr, 1 - par, ph.site, sp, x);
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
// With SPLITW the weights are FP32 values given as hi and lo BF16 operand
// sets (wops, wops + MX_OPS): the lo weights add one more product, so the
// result carries FP32 weights (training) instead of BF16-valued ones.
template <int J, bool SPLITW, typename SI>
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
    if constexpr (SPLITW) {
      const bf16x8 wl = wops[MX_OPS + (t * MX_L1_STEPS + J) * 64 + lane];
#pragma unroll
      for (int a = 0; a < 3; ++a) acc[a][t] = MX_MFMA(wl, bh[a], acc[a][t]);
    }
  }
}

// Layer 1's result in hid (FP32 field, virtual RHS r * 8 + channel): lane
// element e of tile t is hidden row 16 t + 4 g + e = (channel 2 t + g / 2,
// spin 2 (g % 2) + e / 2, re/im e % 2) of colour a at the lane's site.
__device__ __forceinline__ void mx_store_hidden(const Field<float>& hid, int r, int par, int s, int grp,
                                                const floatx4 (&acc)[3][MX_L1_TILES]) {
#pragma unroll
  for (int t = 0; t < MX_L1_TILES; ++t)
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int ch = 2 * t + grp / 2, sp = 2 * (grp % 2) + h, comp = 3 * sp + a;
        float* dst = (float*)&hid.data[hid.cidx(r * PTC_HIDDEN + ch, par, comp / 2, s)] + 2 * (comp & 1);
        dst[0] = acc[a][t][2 * h];
        dst[1] = acc[a][t][2 * h + 1];
      }
}

// One wavefront per 16 sites of one parity and one right-hand side (a tile);
// waves loop over tiles.  The operands of both weight matrices are staged in
// LDS once per workgroup.  Scheduling fences between the K steps keep the
// compiler from hoisting every step's neighbour loads to the top, which
// would take the register count past two waves per SIMD.
//
// MODE 0 (inference): BF16-valued weights, both layers, chi out.
// MODE 1 (training forward): FP32 weights (hi + lo operand sets), both
// layers; layer 1's result is also stored in hid for the gradients.
// MODE 2 (adjoint of layer 2 in layer-1 form): FP32 weights, layer 1 only,
// its result stored in hid.
template <typename SI, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void ptc_mx_kernel(
    Geom g, Links<float> L, Field<SI> in, float* chi, const f4* ops, int n_tiles, Field<float> hid) {
  constexpr bool SPLITW = MODE != 0;
  constexpr int NOPS = MODE == 0 ? MX_OPS : 2 * MX_OPS;
  __shared__ bf16x8 wops[NOPS];
  for (int i = threadIdx.x; i < NOPS; i += blockDim.x) __builtin_memcpy(&wops[i], &ops[i], 16);
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
    mx_l1_step<0, SPLITW>(g, L, in, r, s, par, c, grp, valid, wops, lane, acc);
    MX_SCHED_FENCE
    mx_l1_step<1, SPLITW>(g, L, in, r, s, par, c, grp, valid, wops, lane, acc);
    MX_SCHED_FENCE
    mx_l1_step<2, SPLITW>(g, L, in, r, s, par, c, grp, valid, wops, lane, acc);
    MX_SCHED_FENCE
    if constexpr (MODE != 0) {
      if (valid) mx_store_hidden(hid, r, par, s, grp, acc);
    }
    if constexpr (MODE == 2) continue;
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
          if constexpr (SPLITW) {
            const bf16x8 wl = wops[MX_OPS + (MX_L1_OPS + t * MX_L2_STEPS + j) * 64 + lane];
            o[t] = MX_MFMA(wl, bh[j], o[t]);
          }
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
  hipLaunchKernelGGL((ptc_mx_kernel<SI, 0>), dim3(blocks), dim3(256), 0, st, g, L, in, chi, (const f4*)ops, n_tiles,
                     Field<float>{});
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((ptc_gather_kernel<SO>), dim3((2 * g.vh + 255) / 256, n_rhs), dim3(256), 0, st, g, L, chi, out,
                     n_rhs);
  return hipGetLastError();
}

hipError_t ptc_forward_mx_train(const Geom& g, Links<float> L, Field<double> in, float* chi, Field<float> hid,
                                Field<float> out, const void* ops_split, int n_rhs, hipStream_t st) {
  const int n_tiles = n_rhs * 2 * ((g.vh + 15) / 16);
  int blocks = (n_tiles + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((ptc_mx_kernel<double, 1>), dim3(blocks), dim3(256), 0, st, g, L, in, chi, (const f4*)ops_split,
                     n_tiles, hid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((ptc_gather_kernel<float>), dim3((2 * g.vh + 255) / 256, n_rhs), dim3(256), 0, st, g, L, chi,
                     out, n_rhs);
  return hipGetLastError();
}

hipError_t ptc_adjoint2_mx(const Geom& g, Links<float> L, Field<float> gy, Field<float> gh, const void* ops_adj_split,
                           int n_pairs, hipStream_t st) {
  const int n_tiles = n_pairs * 2 * ((g.vh + 15) / 16);
  int blocks = (n_tiles + 3) / 4;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL((ptc_mx_kernel<float, 2>), dim3(blocks), dim3(256), 0, st, g, L, gy, nullptr,
                     (const f4*)ops_adj_split, n_tiles, gh);
  return hipGetLastError();
}

template hipError_t ptc_forward_mx<double, double>(const Geom&, Links<float>, Field<double>, float*, Field<double>,
                                                   const void*, int, hipStream_t);
template hipError_t ptc_forward_mx<float, float>(const Geom&, Links<float>, Field<float>, float*, Field<float>,
                                                 const void*, int, hipStream_t);

// ------------------------------------------- matrix-core weight gradients
// dW[p][c_o][c_i] (complex 4x4 spin matrix [s_o][s_i]) is a sum over pairs
// k, sites n and colours a of A(n)_{s_o, a} conj(B(n)_{s_i, a}), A on the
// output side and B on the input side, one of them transported:
//   layer 1:  A = gh (8 channels),          B = T_p x (9 paths, 1 channel);
//   layer 2:  A = T_q gy (9 paths, q = pbar: T_p^+ = T_pbar), B = h (8 channels).
// Per colour and pair this is a real matrix product over K = (site, re/im):
// C[(a, ri)][b] with a = (path or channel, s_o) and b = (path or channel, s_i),
//   C[(a, re)][b] = sum (A_re B_re + A_im B_im),   C[(a, im)][b] = sum (A_im B_re - A_re B_im),
// so the A row (a, re) carries (A_re, A_im) and the row (a, im) carries
// (A_im, -A_re) against the B column's (B_re, B_im).
//
// A workgroup walks (16-site tile, pair) units: its threads load the
// untransported field and transport the other one for the tile into LDS,
// then each wavefront runs the 16x16x32 BF16 matrix instruction for its
// share of the C tiles, K = 16 sites x (re, im) per colour.  Both operands
// are FP32 values split as hi + lo (as in the forward pass); hi*hi, hi*lo
// and lo*hi are accumulated in FP32 (the dropped lo*lo is below 2^-16 of the
// product).  Every workgroup stores its C, and a fixed-order FP64 reduction
// over the workgroups gives the gradient.
constexpr int WG_SITES = 16;

template <int ROWS>
struct WgVals {
  cpx<float> v[ROWS][3][WG_SITES];  // [row = (path or channel, spin)][colour][site]
};

// The untransported side: rows (c, s) of the C-channel FP32 field f for
// virtual RHS k * C + c, one 16-byte chunk (two colour components) per
// item, loaded in one call and stored to LDS in the next (the loads of the
// next pair are in flight while the current pair's matrix products run).
template <int C>
struct WgPlainRegs {
  static constexpr int ITEMS = (C * 6 * WG_SITES + 255) / 256;
  f4 q[ITEMS];
};
template <int C>
__device__ __forceinline__ void wg_plain_load(const Geom& g, const Field<float>& f, int k, int par, int s0,
                                              WgPlainRegs<C>& R) {
#pragma unroll
  for (int j = 0; j < WgPlainRegs<C>::ITEMS; ++j) {
    const int it = threadIdx.x + 256 * j;
    const int site = it % WG_SITES, ch = (it / WG_SITES) % 6, c = it / (6 * WG_SITES);
    const int s = s0 + site;
    R.q[j] = f4{0.f, 0.f, 0.f, 0.f};
    if (it < C * 6 * WG_SITES && s < g.vh) R.q[j] = f.data[f.cidx(k * C + c, par, ch, s)];
  }
}
template <int C, int ROWS>
__device__ __forceinline__ void wg_plain_store(const WgPlainRegs<C>& R, WgVals<ROWS>& out) {
  static_assert(ROWS == 4 * C, "rows");
#pragma unroll
  for (int j = 0; j < WgPlainRegs<C>::ITEMS; ++j) {
    const int it = threadIdx.x + 256 * j;
    if (it >= C * 6 * WG_SITES) continue;
    const int site = it % WG_SITES, ch = (it / WG_SITES) % 6, c = it / (6 * WG_SITES);
    const int c0 = 2 * ch, c1 = 2 * ch + 1;  // colour components 3 s + a
    out.v[c * 4 + c0 / 3][c0 % 3][site] = cpx<float>{R.q[j].x, R.q[j].y};
    out.v[c * 4 + c1 / 3][c1 % 3][site] = cpx<float>{R.q[j].z, R.q[j].w};
  }
}

// The transported side: rows (q, s) of T_q f for the one-channel field f,
// one item per (path, site, spin), 576 items over the 256 threads.  Per tile
// the items' neighbours are found once and the tile's links (third row
// rebuilt) staged in LDS; per pair an item loads its neighbour's spin
// (next pair's loads in flight as above) and multiplies by the link.
constexpr int WG_TITEMS = (PTC_PATHS * WG_SITES * 4 + 255) / 256;
struct WgLinks {
  cpx<float> u[PTC_PATHS - 1][WG_SITES][9];  // path q = 1..8 at [q - 1]
};
struct WgTransItem {
  int nsite, npar;  // neighbour (or the site itself for q = 0)
  float sgn;        // 0 across a Schroedinger-functional boundary or past the tile
};
struct WgTransRegs {
  cpx<float> x[WG_TITEMS][3];
};

__device__ __forceinline__ void wg_trans_setup(const Geom& g, const Links<float>& L, int par, int s0, WgLinks& lk,
                                               WgTransItem (&items)[WG_TITEMS]) {
  for (int it = threadIdx.x; it < (PTC_PATHS - 1) * WG_SITES; it += blockDim.x) {
    const int site = it % WG_SITES, q = 1 + it / WG_SITES;
    const int s = s0 + site;
    cpx<float> u[9];
#pragma unroll
    for (int e = 0; e < 9; ++e) u[e] = {0.f, 0.f};
    if (s < g.vh) {
      const Coords c = site_coords(g, s, par);
      const int mu = q <= 4 ? q - 1 : q - 5;
      const PathHop ph = path_hop(g, c, s, par, mu, q <= 4);
      load_link(L, ph.link_par, mu, ph.link_site, u);
    }
#pragma unroll
    for (int e = 0; e < 9; ++e) lk.u[q - 1][site][e] = u[e];
  }
#pragma unroll
  for (int j = 0; j < WG_TITEMS; ++j) {
    const int it = threadIdx.x + 256 * j;
    const int site = it % WG_SITES, q = it / (4 * WG_SITES);
    const int s = s0 + site;
    WgTransItem t{s < g.vh ? s : 0, par, 0.f};
    if (it < PTC_PATHS * WG_SITES * 4 && s < g.vh) {
      t.sgn = 1.f;
      if (q > 0) {
        const Coords c = site_coords(g, s, par);
        const int mu = q <= 4 ? q - 1 : q - 5;
        const PathHop ph = path_hop(g, c, s, par, mu, q <= 4);
        t.nsite = ph.site;
        t.npar = 1 - par;
        t.sgn = ph.ok ? ph.sgn : 0.f;
      }
    }
    items[j] = t;
  }
}

template <typename SF>
__device__ __forceinline__ void wg_trans_load(const Field<SF>& f, int k, const WgTransItem (&items)[WG_TITEMS],
                                              WgTransRegs& R) {
#pragma unroll
  for (int j = 0; j < WG_TITEMS; ++j) {
    const int it = threadIdx.x + 256 * j;
    const int sp = (it / WG_SITES) & 3;
#pragma unroll
    for (int b = 0; b < 3; ++b) R.x[j][b] = {0.f, 0.f};
    if (items[j].sgn != 0.f) load_spin_any(f, k, items[j].npar, items[j].nsite, sp, R.x[j]);
  }
}

template <int ROWS>
__device__ __forceinline__ void wg_trans_store(const WgTransRegs& R, const WgTransItem (&items)[WG_TITEMS],
                                               const WgLinks& lk, WgVals<ROWS>& out) {
  static_assert(ROWS == 4 * PTC_PATHS, "rows");
#pragma unroll
  for (int j = 0; j < WG_TITEMS; ++j) {
    const int it = threadIdx.x + 256 * j;
    if (it >= PTC_PATHS * WG_SITES * 4) continue;
    const int site = it % WG_SITES, sp = (it / WG_SITES) & 3, q = it / (4 * WG_SITES);
    const float sg = items[j].sgn;
    cpx<float> y[3];
    if (q == 0) {
#pragma unroll
      for (int a = 0; a < 3; ++a) y[a] = sg * R.x[j][a];
    } else {
      const cpx<float>* u = lk.u[q - 1][site];
      const bool fwd = q <= 4;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        cpx<float> acc = {0.f, 0.f};
#pragma unroll
        for (int b = 0; b < 3; ++b) acc = acc + (fwd ? cmul(u[3 * a + b], R.x[j][b]) : cjmul(u[3 * b + a], R.x[j][b]));
        y[a] = sg * acc;
      }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) out.v[q * 4 + sp][a][site] = y[a];
  }
}

// The operands of one C tile for colour a: lane l, group gp = l / 16,
// element i: A row 16 mt + l % 16 and B column 16 nt + l % 16, both at
// k = 8 gp + i = (site 4 gp + i / 2, re/im i % 2).
template <int AR, int BC>
__device__ __forceinline__ void wg_operands(const WgVals<AR>& A, const WgVals<BC>& B, int mt, int nt, int a,
                                            int lane, bf16x8& ah, bf16x8& al, bf16x8& bh, bf16x8& bl) {
  const int m = 16 * mt + (lane & 15), n = 16 * nt + (lane & 15), gp = lane >> 4;
  const int ar = m >> 1, ri = m & 1;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int site = 4 * gp + j;
    cpx<float> z = {0.f, 0.f}, b = {0.f, 0.f};
    if (ar < AR) z = A.v[ar][a][site];
    if (n < BC) b = B.v[n][a][site];
    const float a0 = ri == 0 ? z.re : z.im, a1 = ri == 0 ? z.im : -z.re;
    __bf16 hi, lo;
    split_bf16(a0, hi, lo);
    ah[2 * j] = hi;
    al[2 * j] = lo;
    split_bf16(a1, hi, lo);
    ah[2 * j + 1] = hi;
    al[2 * j + 1] = lo;
    split_bf16(b.re, hi, lo);
    bh[2 * j] = hi;
    bl[2 * j] = lo;
    split_bf16(b.im, hi, lo);
    bh[2 * j + 1] = hi;
    bl[2 * j + 1] = lo;
  }
}

template <int LAYER, typename SX>
__device__ __forceinline__ Field<float> wg_plain_field(const Field<SX>& x, const Field<float>& gf) {
  if constexpr (LAYER == 1) return gf;
  else return x;  // layer 2: x is the FP32 hidden field
}

// LAYER 1: A = gh (Field<float>, 8 channels), B = T_p x (Field<SX>).
// LAYER 2: A = T_q gy (Field<float>), B = h (Field<float>, 8 channels).
// A workgroup takes 16-site tiles (grid-stride) and walks the pairs inside
// a tile with two LDS operand buffers: the loads of pair k + 1 are issued
// before pair k's matrix products, and stored after them.
// part[(blk * MT * 16 + m) * NT * 16 + n] = this workgroup's C[m][n].
template <int LAYER, typename SX>
__global__ __launch_bounds__(256) void ptc_wgrad_mx_kernel(Geom g, Links<float> L, Field<SX> x, Field<float> gf,
                                                           int n_pairs, float* part) {
  constexpr int AR = LAYER == 1 ? 4 * PTC_HIDDEN : 4 * PTC_PATHS;  // complex A rows
  constexpr int BC = LAYER == 1 ? 4 * PTC_PATHS : 4 * PTC_HIDDEN;  // B columns
  constexpr int MT = (2 * AR + 15) / 16, NT = (BC + 15) / 16, CT = MT * NT;
  constexpr int CPW = (CT + 3) / 4;  // C tiles per wavefront
  __shared__ WgVals<AR> A[2];
  __shared__ WgVals<BC> B[2];
  __shared__ WgLinks lk;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  floatx4 acc[CPW];
#pragma unroll
  for (int i = 0; i < CPW; ++i) acc[i] = floatx4{0.f, 0.f, 0.f, 0.f};
  const int tpp = (g.vh + WG_SITES - 1) / WG_SITES;
  // the plain side is gh (layer 1) or h (layer 2), both FP32 with 8 channels;
  // the transported side is x (layer 1) or gy (layer 2)
  const Field<float> plain = wg_plain_field<LAYER>(x, gf);
  WgPlainRegs<PTC_HIDDEN> pr;
  WgTransRegs tr;
  WgTransItem items[WG_TITEMS];
  for (int tile = blockIdx.x; tile < 2 * tpp; tile += gridDim.x) {
    const int par = tile / tpp, s0 = (tile - par * tpp) * WG_SITES;
    __syncthreads();  // the previous tile's last products have read lk and the buffers
    wg_trans_setup(g, L, par, s0, lk, items);
    wg_plain_load<PTC_HIDDEN>(g, plain, 0, par, s0, pr);
    if constexpr (LAYER == 1) wg_trans_load(x, 0, items, tr);
    else wg_trans_load(gf, 0, items, tr);
    __syncthreads();  // lk
    for (int k = 0; k < n_pairs; ++k) {
      const int buf = k & 1;
      if constexpr (LAYER == 1) {
        wg_plain_store<PTC_HIDDEN>(pr, A[buf]);
        wg_trans_store(tr, items, lk, B[buf]);
      } else {
        wg_trans_store(tr, items, lk, A[buf]);
        wg_plain_store<PTC_HIDDEN>(pr, B[buf]);
      }
      __syncthreads();  // buffer buf complete; buffer 1 - buf no longer read
      if (k + 1 < n_pairs) {
        wg_plain_load<PTC_HIDDEN>(g, plain, k + 1, par, s0, pr);
        if constexpr (LAYER == 1) wg_trans_load(x, k + 1, items, tr);
        else wg_trans_load(gf, k + 1, items, tr);
      }
#pragma unroll
      for (int i = 0; i < CPW; ++i) {
        const int ct = wave + 4 * i;
        if (ct < CT) {
          const int mt = ct / NT, nt = ct - mt * NT;
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            bf16x8 ah, al, bh, bl;
            wg_operands<AR, BC>(A[buf], B[buf], mt, nt, a, lane, ah, al, bh, bl);
            acc[i] = MX_MFMA(ah, bh, acc[i]);
            acc[i] = MX_MFMA(ah, bl, acc[i]);
            acc[i] = MX_MFMA(al, bh, acc[i]);
          }
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < CPW; ++i) {
    const int ct = wave + 4 * i;
    if (ct < CT) {
      const int mt = ct / NT, nt = ct - mt * NT;
      const int n = 16 * nt + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = 16 * mt + 4 * (lane >> 4) + e;
        part[((long)blockIdx.x * MT * 16 + m) * (NT * 16) + n] = acc[i][e];
      }
    }
  }
}

// grad[(p c_out + c_o) c_in + c_i][2 (4 s_o + s_i) + ri] = sum over workgroups
// of C[(a, ri)][b], in a fixed order (FP64); one wavefront per entry.
template <int LAYER>
__global__ void ptc_wgrad_mx_reduce_kernel(const float* part, int nblk, double* grad) {
  constexpr int AR = LAYER == 1 ? 4 * PTC_HIDDEN : 4 * PTC_PATHS;
  constexpr int BC = LAYER == 1 ? 4 * PTC_PATHS : 4 * PTC_HIDDEN;
  constexpr int MT = (2 * AR + 15) / 16, NT = (BC + 15) / 16;
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= 2 * AR * BC) return;
  const int m = w / BC, n = w - m * BC;
  double v = 0.0;
  for (int j = lane; j < nblk; j += 64) v += (double)part[((long)j * MT * 16 + m) * (NT * 16) + n];
  v = wave_sum(v);
  if (lane != 0) return;
  const int ar = m >> 1, ri = m & 1;
  const int so = ar & 3, si = n & 3;
  int idx;
  if constexpr (LAYER == 1) {
    const int co = ar >> 2, p = n >> 2;  // W1[p][co] (c_in = 1)
    idx = p * PTC_HIDDEN + co;
  } else {
    const int q = ar >> 2, ci = n >> 2;  // W2[p][ci] with q = pbar (c_out = 1)
    const int p = q == 0 ? 0 : (q <= 4 ? q + 4 : q - 4);
    idx = p * PTC_HIDDEN + ci;
  }
  grad[(long)idx * 32 + 2 * (4 * so + si) + ri] = v;
}

size_t ptc_wgrad_mx_part_floats(int nblk) {
  constexpr int M1 = ((2 * 4 * PTC_HIDDEN + 15) / 16) * 16, N1 = ((4 * PTC_PATHS + 15) / 16) * 16;
  constexpr int M2 = ((2 * 4 * PTC_PATHS + 15) / 16) * 16, N2 = ((4 * PTC_HIDDEN + 15) / 16) * 16;
  return (size_t)nblk * (M1 * N1 > M2 * N2 ? M1 * N1 : M2 * N2);
}

template <int LAYER, typename SX>
hipError_t ptc_weight_grad_mx(const Geom& g, Links<float> L, Field<SX> x, Field<float> gf, int n_pairs, int nblk,
                              float* part, double* grad, hipStream_t st) {
  hipLaunchKernelGGL((ptc_wgrad_mx_kernel<LAYER, SX>), dim3(nblk), dim3(256), 0, st, g, L, x, gf, n_pairs, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  constexpr int AR = LAYER == 1 ? 4 * PTC_HIDDEN : 4 * PTC_PATHS;
  constexpr int BC = LAYER == 1 ? 4 * PTC_PATHS : 4 * PTC_HIDDEN;
  const int waves = 2 * AR * BC;
  hipLaunchKernelGGL((ptc_wgrad_mx_reduce_kernel<LAYER>), dim3((waves + 3) / 4), dim3(256), 0, st, part, nblk, grad);
  return hipGetLastError();
}

template hipError_t ptc_weight_grad_mx<1, double>(const Geom&, Links<float>, Field<double>, Field<float>, int, int,
                                                  float*, double*, hipStream_t);
template hipError_t ptc_weight_grad_mx<2, float>(const Geom&, Links<float>, Field<float>, Field<float>, int, int,
                                                 float*, double*, hipStream_t);

}  // namespace mfq
