// Restarted flexible GMRES (right preconditioning) for all RHS at once, with
// the learned PTC network as the preconditioner and plain CG as the fallback.
//
// Per RHS, a cycle of at most m steps builds an orthonormal basis v_j, the
// preconditioned directions z_j = M v_j and the Hessenberg matrix H of
// A z_j = sum_i H_ij v_i (classical Gram-Schmidt applied twice, FP64 dot
// products), rotates H to triangular form with complex Givens rotations on
// the device, and updates x += Z y with H y = g at the end of the cycle.  The
// next cycle restarts from the FP64 true residual.  The host syncs once per
// cycle.  If a cycle fails to reduce the true residual, or produces NaN, the
// solve falls back to CG on the remaining residual.
#include <math.h>
#include <string.h>

#include <chrono>

#include "handle.h"
#include "hop_impl.h"

namespace mfq {

constexpr int GM_MAXM = 32;

struct GmState {
  double hr[(GM_MAXM + 1) * GM_MAXM], hi[(GM_MAXM + 1) * GM_MAXM];  // H(i, j) at j * (M + 1) + i
  double csr[GM_MAXM], csi[GM_MAXM], snr[GM_MAXM], sni[GM_MAXM];
  double gr[GM_MAXM + 1], gi[GM_MAXM + 1];
  double yr[GM_MAXM], yi[GM_MAXM];
  double cr[GM_MAXM + 1], ci[GM_MAXM + 1];  // Gram-Schmidt coefficients of the current pass
  double bnorm2, rtrue2, wnorm;
  double w2;   // |w|^2 before the first Gram-Schmidt pass
  int k, active, done, iters, cycles;
  int reorth;  // the second Gram-Schmidt pass is needed for this step
};

#define GM_LANE                                                    \
  const int q = blockIdx.x * blockDim.x + threadIdx.x;             \
  const int r = blockIdx.y;                                        \
  const bool valid = q < 2 * g.vh;                                 \
  const int par = q >= g.vh ? 1 : 0;                               \
  const int s = q - par * g.vh;

__device__ __forceinline__ void block_sum2(double a, double b, double* part_a, double* part_b) {
  __shared__ double ws[2][4];
  a = wave_sum(a);
  b = wave_sum(b);
  if ((threadIdx.x & 63) == 0) {
    ws[0][threadIdx.x >> 6] = a;
    ws[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *part_a = ((ws[0][0] + ws[0][1]) + ws[0][2]) + ws[0][3];
    *part_b = ((ws[1][0] + ws[1][1]) + ws[1][2]) + ws[1][3];
  }
  __syncthreads();
}

// <v_l, w> for l < NV, and with `first` also |w|^2 as entry NV: partials
// part[((r * (NV + 1) + l) * nblk + blk) * 2 + {re, im}].  All NV dot
// products accumulate in registers (the basis vectors' loads issue together)
// and meet in one workgroup reduction.  The second pass runs only for the RHS
// whose first pass asked for it (the whole workgroup belongs to one RHS, so it
// returns together).
template <int NV, typename S>
__global__ __launch_bounds__(256) void gm_multidot_kernel(Geom g, Field<S> V, size_t vstride, Field<S> w,
                                                          int n_rhs, double* part, int first, const GmState* st) {
  GM_LANE
  if (!first && !st[r].reorth) return;
  constexpr int NVAL = 2 * NV + 1;
  double acc[NVAL];
#pragma unroll
  for (int i = 0; i < NVAL; ++i) acc[i] = 0.0;
  if (valid) {
    Spinor<double> ww;
    load_spinor(w, r, par, s, ww);
#pragma unroll
    for (int k = 0; k < 12; ++k) acc[2 * NV] += norm2(ww.v[k]);
#pragma unroll
    for (int l = 0; l < NV; ++l) {
      Field<S> vl = V;
      vl.data += l * vstride;
      Spinor<double> vv;
      load_spinor(vl, r, par, s, vv);
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        const cpx<double> d = cjmul(vv.v[k], ww.v[k]);
        acc[2 * l] += d.re;
        acc[2 * l + 1] += d.im;
      }
    }
  }
  __shared__ double ws[4][NVAL];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NVAL; ++i) {
    const double v = wave_sum(acc[i]);
    if (lane == 0) ws[wv][i] = v;
  }
  __syncthreads();
  const int i = threadIdx.x;
  if (i < 2 * NV || (first && i == 2 * NV)) {
    const double v = ((ws[0][i] + ws[1][i]) + ws[2][i]) + ws[3][i];
    const int l = i / 2;  // i = 2 NV gives l = NV, the |w|^2 entry
    double* base = part + (((long)r * (NV + 1) + l) * gridDim.x + blockIdx.x) * 2;
    if (i < 2 * NV) {
      base[i % 2] = v;
    } else {
      base[0] = v;
      base[1] = 0.0;
    }
  }
}

// coefficients c_l = sum of partials; H(:, j) += c (accumulate over passes).
// One wavefront per (RHS, l); the first pass also reduces |w|^2 (l = nv).
__global__ void gm_dots_finish_kernel(const double* part, int nblk, int nv, int n_rhs, GmState* st, int j, int first) {
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int nl = nv + (first ? 1 : 0);
  if (w >= n_rhs * nl) return;
  const int r = w / nl, l = w % nl;
  if (!first && !st[r].reorth) return;
  double re = 0.0, im = 0.0;
  const double* p = part + ((long)r * (nv + 1) + l) * nblk * 2;
  for (int b = lane; b < nblk; b += 64) {
    re += p[2 * b];
    im += p[2 * b + 1];
  }
  re = wave_sum(re);
  im = wave_sum(im);
  if (lane == 0) {
    GmState& S = st[r];
    if (l == nv) {  // first pass: |w|^2 before the projection
      S.w2 = re;
      return;
    }
    S.cr[l] = re;
    S.ci[l] = im;
    const int idx = j * (GM_MAXM + 1) + l;
    if (first) {
      S.hr[idx] = re;
      S.hi[idx] = im;
    } else {
      S.hr[idx] += re;
      S.hi[idx] += im;
    }
  }
}

// w -= sum_l c_l v_l (l < NV, unrolled so that the loads issue together).
// After the first pass, workgroup 0 of each RHS decides whether the second
// pass is needed: the projected norm |w'|^2 = |w|^2 - sum |c_l|^2 below
// 1 % of |w|^2 (|w'| < 0.1 |w|) means cancellation has eaten the
// orthogonality and the pass is repeated.  (Kahan's 0.7 fires on nearly
// every step once the preconditioner is good, since A z_j then lies almost
// in the span of the basis; each cycle restarts from the FP64 true residual,
// so lost orthogonality could only cost iterations.)  No other workgroup of
// this launch reads the flag.
template <int NV, typename S>
__global__ __launch_bounds__(256) void gm_multiaxpy_kernel(Geom g, Field<S> V, size_t vstride, Field<S> w,
                                                           int n_rhs, GmState* st, int first) {
  GM_LANE
  if (!first && !st[r].reorth) return;
  if (first && blockIdx.x == 0 && threadIdx.x == 0) {
    double c2 = 0.0;
    for (int l = 0; l < NV; ++l) c2 += st[r].cr[l] * st[r].cr[l] + st[r].ci[l] * st[r].ci[l];
    const double w2 = st[r].w2;
    st[r].reorth = !(w2 - c2 > 0.01 * w2);
  }
  if (!valid) return;
  Spinor<double> ww;
  load_spinor(w, r, par, s, ww);
#pragma unroll
  for (int l = 0; l < NV; ++l) {
    const cpx<double> c = {st[r].cr[l], st[r].ci[l]};
    Field<S> vl = V;
    vl.data += l * vstride;
    Spinor<double> vv;
    load_spinor(vl, r, par, s, vv);
#pragma unroll
    for (int k = 0; k < 12; ++k) ww.v[k] = ww.v[k] - cmul(c, vv.v[k]);
  }
  store_spinor(w, r, par, s, ww);
}

#define GM_NV_CASES(X)                                                                                              \
  X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) X(20) \
  X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)
static_assert(GM_MAXM == 32, "one multidot / multiaxpy instance per basis size 1..GM_MAXM");

template <typename SV>
hipError_t launch_multidot(int nv, dim3 grid, dim3 blk, hipStream_t st, const Geom& g, Field<SV> V,
                           size_t vstride, Field<SV> w, int n, double* part, int first, const GmState* S) {
  switch (nv) {
#define GM_DOT(N)                                                                                                \
  case N:                                                                                                        \
    hipLaunchKernelGGL((gm_multidot_kernel<N, SV>), grid, blk, 0, st, g, V, vstride, w, n, part, first, S);      \
    break;
    GM_NV_CASES(GM_DOT)
#undef GM_DOT
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename SV>
hipError_t launch_multiaxpy(int nv, dim3 grid, dim3 blk, hipStream_t st, const Geom& g, Field<SV> V,
                            size_t vstride, Field<SV> w, int n, GmState* S, int first) {
  switch (nv) {
#define GM_AXPY(N)                                                                                               \
  case N:                                                                                                        \
    hipLaunchKernelGGL((gm_multiaxpy_kernel<N, SV>), grid, blk, 0, st, g, V, vstride, w, n, S, first);           \
    break;
    GM_NV_CASES(GM_AXPY)
#undef GM_AXPY
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename S>
__global__ __launch_bounds__(256) void gm_norm_kernel(Geom g, Field<S> w, int n_rhs, double* part) {
  GM_LANE
  double v = 0.0;
  if (valid) {
    Spinor<double> ww;
    load_spinor(w, r, par, s, ww);
#pragma unroll
    for (int k = 0; k < 12; ++k) v += norm2(ww.v[k]);
  }
  double* base = part + ((long)r * gridDim.x + blockIdx.x) * 2;
  block_sum2(v, 0.0, base, base + 1);
}

// which = 0: |w| -> H(j+1, j) and S.wnorm; which = 1: |b|^2 -> S.bnorm2,
// beta = |b|, g = (beta, 0, ...); which = 2: true residual |r|^2 -> rtrue2,
// done flag, restart g = (|r|, 0, ...)
__global__ void gm_norm_finish_kernel(const double* part, int nblk, int n_rhs, GmState* st, int j, int which,
                                      double tol2) {
  const int w = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (w >= n_rhs) return;
  double v = 0.0;
  const double* p = part + (long)w * nblk * 2;
  for (int b = lane; b < nblk; b += 64) v += p[2 * b];
  v = wave_sum(v);
  if (lane != 0) return;
  GmState& S = st[w];
  if (which == 0) {
    S.wnorm = sqrt(v);
    S.hr[j * (GM_MAXM + 1) + j + 1] = S.wnorm;
    S.hi[j * (GM_MAXM + 1) + j + 1] = 0.0;
  } else {
    if (which == 1) {
      S.bnorm2 = v;
      S.iters = 0;
      S.cycles = 0;
      S.done = v > 0.0 ? 0 : 1;
    } else {
      S.cycles += 1;
      if (!S.done && v <= tol2 * S.bnorm2) S.done = 1;
    }
    S.rtrue2 = v;
    S.wnorm = sqrt(v);
    for (int i = 0; i <= GM_MAXM; ++i) S.gr[i] = S.gi[i] = 0.0;
    S.gr[0] = S.wnorm;
    S.k = 0;
    S.active = S.done ? 0 : 1;
  }
}

// v_out = w / |w| (|w| from the state); zero if |w| = 0
template <typename SI, typename SO>
__global__ __launch_bounds__(256) void gm_scale_kernel(Geom g, Field<SI> w, Field<SO> vout, int n_rhs,
                                                       const GmState* st) {
  GM_LANE
  if (!valid) return;
  const double nrm = st[r].wnorm;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  Spinor<double> ww;
  load_spinor(w, r, par, s, ww);
#pragma unroll
  for (int k = 0; k < 12; ++k) ww.v[k] = inv * ww.v[k];
  store_spinor(vout, r, par, s, ww);
}

// rotations for column j, one thread per RHS
__global__ void gm_givens_kernel(GmState* st, int n_rhs, int j, int m, double tol2) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rhs) return;
  GmState& S = st[r];
  if (!S.active) return;
  const int col = j * (GM_MAXM + 1);
  for (int l = 0; l < j; ++l) {
    const cpx<double> c = {S.csr[l], S.csi[l]}, sn = {S.snr[l], S.sni[l]};
    const cpx<double> a = {S.hr[col + l], S.hi[col + l]}, b = {S.hr[col + l + 1], S.hi[col + l + 1]};
    const cpx<double> t = cjmul(c, a) + cjmul(sn, b);
    const cpx<double> u = cmul(c, b) - cmul(sn, a);
    S.hr[col + l] = t.re;
    S.hi[col + l] = t.im;
    S.hr[col + l + 1] = u.re;
    S.hi[col + l + 1] = u.im;
  }
  const cpx<double> a = {S.hr[col + j], S.hi[col + j]}, b = {S.hr[col + j + 1], S.hi[col + j + 1]};
  const double den = sqrt(norm2(a) + norm2(b));
  S.iters += 1;
  if (!(den > 0.0) || !isfinite(den)) {  // breakdown: stop this cycle before column j
    S.active = 0;
    return;
  }
  const cpx<double> c = {a.re / den, a.im / den}, sn = {b.re / den, b.im / den};
  S.csr[j] = c.re;
  S.csi[j] = c.im;
  S.snr[j] = sn.re;
  S.sni[j] = sn.im;
  S.hr[col + j] = den;
  S.hi[col + j] = 0.0;
  S.hr[col + j + 1] = 0.0;
  S.hi[col + j + 1] = 0.0;
  const cpx<double> gj = {S.gr[j], S.gi[j]};
  const cpx<double> g1 = -cmul(sn, gj);
  const cpx<double> g0 = cjmul(c, gj);
  S.gr[j] = g0.re;
  S.gi[j] = g0.im;
  S.gr[j + 1] = g1.re;
  S.gi[j + 1] = g1.im;
  S.k = j + 1;
  if (norm2(g1) <= tol2 * S.bnorm2 || j + 1 >= m) S.active = 0;
}

// back substitution H(0:k, 0:k) y = g(0:k), one thread per RHS
__global__ void gm_solve_kernel(GmState* st, int n_rhs) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n_rhs) return;
  GmState& S = st[r];
  for (int i = S.k - 1; i >= 0; --i) {
    cpx<double> acc = {S.gr[i], S.gi[i]};
    for (int l = i + 1; l < S.k; ++l) {
      const cpx<double> h = {S.hr[l * (GM_MAXM + 1) + i], S.hi[l * (GM_MAXM + 1) + i]};
      acc = acc - cmul(h, cpx<double>{S.yr[l], S.yi[l]});
    }
    const double d = S.hr[i * (GM_MAXM + 1) + i];  // real after rotation
    S.yr[i] = acc.re / d;
    S.yi[i] = acc.im / d;
  }
}

// x += sum_{j < k} y_j z_j
template <typename SZ>
__global__ __launch_bounds__(256) void gm_xupdate_kernel(Geom g, Field<SZ> Z, size_t zstride, Field<double> x,
                                                         int n_rhs, const GmState* st) {
  GM_LANE
  if (!valid) return;
  const int k = st[r].k;
  if (k == 0) return;
  Spinor<double> xx;
  load_spinor(x, r, par, s, xx);
  for (int j = 0; j < k; ++j) {
    const cpx<double> y = {st[r].yr[j], st[r].yi[j]};
    Field<SZ> zj = Z;
    zj.data += j * zstride;
    Spinor<double> zz;
    load_spinor(zj, r, par, s, zz);
#pragma unroll
    for (int c = 0; c < 12; ++c) xx.v[c] = xx.v[c] + cmul(y, zz.v[c]);
  }
  store_spinor(x, r, par, s, xx);
}

// a += b (both parities, all RHS)
__global__ __launch_bounds__(256) void gm_add_kernel(Geom g, Field<double> a, Field<double> b, int n_rhs) {
  GM_LANE
  if (!valid) return;
  Spinor<double> x, y;
  load_spinor(a, r, par, s, x);
  load_spinor(b, r, par, s, y);
#pragma unroll
  for (int k = 0; k < 12; ++k) x.v[k] = x.v[k] + y.v[k];
  store_spinor(a, r, par, s, x);
}

}  // namespace mfq

using namespace mfq;

namespace {

template <typename F>
struct FieldElem;
template <typename X>
struct FieldElem<mfq::Field<X>> {
  using type = X;
};

template <typename S>
Field<S> raw_field(const DevBuf& b, const Geom& g) {
  Field<S> f;
  f.data = (typename Store<S>::chunk*)b.ptr;
  f.norm = nullptr;
  f.vh = g.vs;
  return f;
}

}  // namespace

namespace mfq {

// Right-preconditioned FGMRES(m) on D^+D x64 = b64 (packed FP64).  S is the
// precision of the cycle: the basis, the preconditioned directions, the
// operator inside the cycle and the network's input and output (FP64, or
// FP32 with the links' FP32 copy); the solution, the true residual each
// cycle restarts from and the Hessenberg entries (FP64 sums of the dot
// products) are FP64 in both.
//
// The basis and the state stay in the handle between calls, and one restart
// cycle (m Arnoldi steps, the update of x, the FP64 true residual and the
// next v_0) is captured once as a graph and replayed for every cycle: the
// host only reads the per-RHS state between cycles.
template <typename S>
int run_fgmres_t(mfq_handle* h, int n, const mfq_solve_params* P, hipStream_t st, mfq_solve_stats* stats) {
  const Geom& g = h->g;
  Workspace& w = h->ws;
  const int m = P->restart > 0 ? (P->restart < GM_MAXM ? P->restart : GM_MAXM) : 16;
  const bool use_pc = P->precond == MFQ_PC_PTC;
  const double tol2 = P->tol * P->tol;
  using C = typename Store<S>::chunk;
  const size_t fch = field_chunks<S>(g, n);         // chunks of one n-RHS field in the cycle precision
  const size_t fch64 = field_chunks<double>(g, n);  // ... and in FP64
  const int nblk = (2 * g.vh + 255) / 256;
  if (ensure(w.gm_v, fch * (m + 1) * sizeof(C)) || (use_pc && ensure(w.gm_z, fch * m * sizeof(C))) ||
      ensure(w.gm_w, fch * sizeof(C)) || ensure(w.gm_st, sizeof(GmState) * n) ||
      ensure(w.gm_part, sizeof(double) * 2 * (size_t)n * (m + 1) * nblk))
    return fail(MFQ_ERR_NOMEM, "FGMRES workspace");
  std::vector<GmState> host(n);
  const dim3 grid(nblk, n), blk(256);
  GmState* Sg = (GmState*)w.gm_st.ptr;
  double* part = (double*)w.gm_part.ptr;
  Field<S> V = raw_field<S>(w.gm_v, g), W = raw_field<S>(w.gm_w, g);
  // without a preconditioner z_j = v_j: the directions are the basis itself
  Field<S> Z = use_pc ? raw_field<S>(w.gm_z, g) : V;
  Field<double> b64 = w.b64.view(g), x64 = w.x64.view(g), r64 = w.r64.view(g), t64 = w.t64.view(g);
  auto vj = [&](Field<S> base, int j) {
    Field<S> f = base;
    f.data += (size_t)j * fch;
    return f;
  };
  Shape sh64;
  if (int rc0 = fp64_hop_shape(h, n, st, &sh64)) return rc0;
  HopArgs<double, double> a64 = hop_args<double, double>(h, links_d(h), n);
  a64.coef = -h->lat.kappa;
  // the operator inside the cycle: D^+ D in precision S
  Shape sh = sh64;
  Field<S> tS;
  Links<S> LS;
  if constexpr (sizeof(S) == 8) {
    tS = t64;
    LS = links_d(h);
  } else {
    if (int rc0 = fp32_hop_shape(h, n, st, &sh)) return rc0;
    tS = w.ts.view(g);
    LS = links_f(h);
  }
  if (use_pc)
    if (int rc0 = ptc_prepare(h, n, st)) return rc0;
  HopArgs<S, S> a = hop_args<S, S>(h, LS, n);
  a.coef = -h->lat.kappa;
  auto apply_a = [&](Field<S> in, Field<S> out, hipStream_t s) -> int {
    a.in = a.self = in;
    a.out = tS;
    a.dagger = 0;
    a.part = nullptr;
    a.par = 2;
    HIPCHK((launch_hop<S, S>(EPI_D, a, sh, s)));
    a.in = a.self = tS;
    a.out = out;
    a.dagger = 1;
    HIPCHK((launch_hop<S, S>(EPI_D, a, sh, s)));
    return MFQ_OK;
  };
  auto norm_finish = [&](auto f, int j, int which, hipStream_t s) -> int {
    hipLaunchKernelGGL((gm_norm_kernel<typename FieldElem<decltype(f)>::type>), grid, blk, 0, s, g, f, n, part);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(gm_norm_finish_kernel, dim3((n + 3) / 4), dim3(256), 0, s, part, nblk, n, Sg, j, which, tol2);
    return hipGetLastError() == hipSuccess ? MFQ_OK : fail(MFQ_ERR_HIP, "gm_norm_finish");
  };
  // the FP64 true residual r64 = b64 - A x64
  auto true_residual = [&](hipStream_t s) -> int {
    a64.in = a64.self = x64;
    a64.out = t64;
    a64.dagger = 0;
    a64.part = nullptr;
    a64.par = 2;
    HIPCHK((launch_hop<double, double>(EPI_D, a64, sh64, s)));
    a64.in = a64.self = t64;
    a64.bvec = b64;
    a64.r64 = r64;
    a64.dagger = 1;
    HIPCHK((launch_hop<double, double>(EPI_RES, a64, sh64, s)));
    return MFQ_OK;
  };
  // one restart cycle, all on the device
  auto cycle_body = [&](hipStream_t s) -> int {
    int rc;
    for (int j = 0; j < m; ++j) {
      if (use_pc)
        if ((rc = ptc_launch_fields(h, vj(V, j), vj(Z, j), n, s))) return rc;
      if ((rc = apply_a(vj(Z, j), W, s))) return rc;
      // classical Gram-Schmidt; the second pass only where the first lost
      // more than 90 % of |w| (the kernels of that pass return at once for
      // the other RHS)
      for (int pass = 0; pass < 2; ++pass) {
        const int first = pass == 0 ? 1 : 0;
        HIPCHK(launch_multidot<S>(j + 1, grid, blk, s, g, V, fch, W, n, part, first, Sg));
        hipLaunchKernelGGL(gm_dots_finish_kernel, dim3((n * (j + 2) + 3) / 4), dim3(256), 0, s, part, nblk, j + 1,
                           n, Sg, j, first);
        HIPCHK(launch_multiaxpy<S>(j + 1, grid, blk, s, g, V, fch, W, n, Sg, first));
      }
      if ((rc = norm_finish(W, j, 0, s))) return rc;
      hipLaunchKernelGGL((gm_scale_kernel<S, S>), grid, blk, 0, s, g, W, vj(V, j + 1), n, Sg);
      hipLaunchKernelGGL(gm_givens_kernel, dim3((n + 63) / 64), dim3(64), 0, s, Sg, n, j, m, tol2);
      HIPCHK(hipGetLastError());
    }
    hipLaunchKernelGGL(gm_solve_kernel, dim3((n + 63) / 64), dim3(64), 0, s, Sg, n);
    hipLaunchKernelGGL((gm_xupdate_kernel<S>), grid, blk, 0, s, g, Z, fch, x64, n, Sg);
    // true residual r = b - A x (FP64), restart v_0 = r / |r|
    if ((rc = true_residual(s))) return rc;
    if ((rc = norm_finish(r64, 0, 2, s))) return rc;
    hipLaunchKernelGGL((gm_scale_kernel<double, S>), grid, blk, 0, s, g, r64, vj(V, 0), n, Sg);
    HIPCHK(hipGetLastError());
    return MFQ_OK;
  };
  hipGraphExec_t cycle_exec = nullptr;
  if (P->use_graph) {
    const PtcState* pc = use_pc ? h->ptc : nullptr;
    std::vector<uintptr_t> key = {(uintptr_t)0x464d5247u, (uintptr_t)sizeof(S), (uintptr_t)n, (uintptr_t)m,
                                  (uintptr_t)use_pc, (uintptr_t)V.data, (uintptr_t)Z.data, (uintptr_t)W.data,
                                  (uintptr_t)Sg, (uintptr_t)part, (uintptr_t)b64.data, (uintptr_t)x64.data,
                                  (uintptr_t)r64.data, (uintptr_t)t64.data, (uintptr_t)tS.data,
                                  (uintptr_t)LS.data, (uintptr_t)a64.links.data,
                                  (uintptr_t)(pc ? pc->chi.ptr : nullptr), (uintptr_t)(pc ? pc->ops.ptr : nullptr),
                                  bits(tol2), bits(h->lat.kappa), (uintptr_t)sh.sb, (uintptr_t)sh.nr,
                                  (uintptr_t)sh.xcd, (uintptr_t)sh.tc, (uintptr_t)sh.ds, (uintptr_t)sh64.sb,
                                  (uintptr_t)sh64.nr, (uintptr_t)sh64.xcd, (uintptr_t)sh64.tc, (uintptr_t)sh64.ds};
    for (auto& e : h->graphs)
      if (e.key == key) cycle_exec = e.exec;
    if (!cycle_exec) {
      if (h->graphs.size() >= 24) drop_graphs(h);
      GraphEntry e;
      e.key = key;
      HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
      const int rc2 = cycle_body(h->cap_stream);
      hipError_t ec = hipStreamEndCapture(h->cap_stream, &e.graph);
      if (rc2 != MFQ_OK) {
        if (e.graph) (void)hipGraphDestroy(e.graph);
        return rc2;
      }
      HIPCHK(ec);
      if ((ec = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0)) != hipSuccess) {
        (void)hipGraphDestroy(e.graph);
        return fail_hip(ec, "FGMRES cycle graph");
      }
      h->graphs.push_back(e);
      cycle_exec = e.exec;
    }
  }
  int rc;
  // x = 0, r = b, v_0 = b / |b|
  HIPCHK(hipMemsetAsync(w.x64.data.ptr, 0, fch64 * sizeof(d2), st));
  if ((rc = norm_finish(b64, 0, 1, st))) return rc;
  hipLaunchKernelGGL((gm_scale_kernel<double, S>), grid, blk, 0, st, g, b64, vj(V, 0), n, Sg);
  const int max_cycles = (P->max_iter + m - 1) / m;
  double prev_worst = 1e300;
  bool fell_back = false;
  int status = MFQ_OK;
  for (int cycle = 0;; ++cycle) {
    if (cycle_exec) {
      HIPCHK(hipGraphLaunch(cycle_exec, st));
    } else if ((rc = cycle_body(st))) {
      return rc;
    }
    HIPCHK(hipMemcpyAsync(host.data(), Sg, sizeof(GmState) * n, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    bool all_done = true, bad = false;
    double worst = 0.0;
    for (int r = 0; r < n; ++r) {
      all_done = all_done && host[r].done;
      if (!isfinite(host[r].rtrue2)) bad = true;
      if (!host[r].done && host[r].bnorm2 > 0) {
        const double rel = sqrt(host[r].rtrue2 / host[r].bnorm2);
        if (rel > worst) worst = rel;
      }
    }
    if (all_done) break;
    // stagnation: a whole cycle that does not reduce the worst residual by 5%
    if (bad || worst > 0.95 * prev_worst || cycle + 1 >= max_cycles) {
      if (cycle + 1 >= max_cycles && !bad && worst <= 0.95 * prev_worst) {
        status = MFQ_NOT_CONVERGED;
        break;
      }
      fell_back = true;
      break;
    }
    prev_worst = worst;
  }
  int cg_iters = 0;
  if (fell_back) {
    // CG on the remaining residual, A e = r with r = b - A x, then x += e.
    // If the preconditioned solve produced NaN, CG starts again from x = 0.
    if (ensure(w.gm_xsave, fch64 * sizeof(d2)) || ensure(w.gm_bsave, fch64 * sizeof(d2)))
      return fail(MFQ_ERR_NOMEM, "FGMRES fallback workspace");
    bool bad = false;
    for (int r = 0; r < n; ++r) bad = bad || !isfinite(host[r].rtrue2);
    if (bad) {
      HIPCHK(hipMemsetAsync(w.x64.data.ptr, 0, fch64 * sizeof(d2), st));
      HIPCHK(hipMemcpyAsync(r64.data, b64.data, fch64 * sizeof(d2), hipMemcpyDeviceToDevice, st));
    }
    // tolerance for the residual system so that |b - A x| <= tol |b| for
    // every RHS: tol * min_i |b_i| / |r_i|
    double ratio = 1.0;
    for (int r = 0; r < n; ++r)
      if (!bad && host[r].rtrue2 > 0 && host[r].bnorm2 > 0)
        ratio = fmin(ratio, sqrt(host[r].bnorm2 / host[r].rtrue2));
    HIPCHK(hipMemcpyAsync(w.gm_xsave.ptr, w.x64.data.ptr, fch64 * sizeof(d2), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(w.gm_bsave.ptr, w.b64.data.ptr, fch64 * sizeof(d2), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(w.b64.data.ptr, r64.data, fch64 * sizeof(d2), hipMemcpyDeviceToDevice, st));
    mfq_solve_params Q = *P;
    Q.precond = MFQ_PC_NONE;
    Q.prec = MFQ_PREC_FP64;
    Q.tol = fmax(fmin(P->tol * ratio, 0.5), 1e-15);
    std::vector<mfq_solve_stats> cst(n);
    rc = solve_packed(h, n, &Q, st, cst.data());
    if (rc < 0) return rc;
    for (int r = 0; r < n; ++r) cg_iters = cg_iters > cst[r].iters ? cg_iters : cst[r].iters;
    hipLaunchKernelGGL(gm_add_kernel, grid, blk, 0, st, g, x64, raw_field<double>(w.gm_xsave, g), n);
    HIPCHK(hipMemcpyAsync(w.b64.data.ptr, w.gm_bsave.ptr, fch64 * sizeof(d2), hipMemcpyDeviceToDevice, st));
    // final FP64 true residual against the original right-hand side
    if ((rc = true_residual(st))) return rc;
    if ((rc = norm_finish(r64, 0, 2, st))) return rc;
    HIPCHK(hipMemcpyAsync(host.data(), Sg, sizeof(GmState) * n, hipMemcpyDeviceToHost, st));
    status = MFQ_FELL_BACK;
    for (int r = 0; r < n; ++r)
      if (!host[r].done) status = MFQ_NOT_CONVERGED;
  }
  HIPCHK(hipStreamSynchronize(st));
  for (int r = 0; r < n; ++r) {
    if (stats) {
      stats[r].iters = host[r].iters + cg_iters;
      stats[r].reliable_updates = host[r].cycles;
      stats[r].true_rel_resid = host[r].bnorm2 > 0 ? sqrt(host[r].rtrue2 / host[r].bnorm2) : 0.0;
      stats[r].status = host[r].done ? (fell_back ? MFQ_FELL_BACK : MFQ_OK) : MFQ_NOT_CONVERGED;
    }
  }
  return status;
}

// FGMRES with the cycle in FP64 (prec FP64) or FP32 (otherwise).
int run_fgmres(mfq_handle* h, int n, const mfq_solve_params* P, hipStream_t st, mfq_solve_stats* stats) {
  if (P->prec == MFQ_PREC_FP64) return run_fgmres_t<double>(h, n, P, st, stats);
  return run_fgmres_t<float>(h, n, P, st, stats);
}

}  // namespace mfq
