// Block conjugate gradients on D^+D (O'Leary): the n right-hand sides share
// one Krylov space, so each RHS's iterate minimises the A-norm of its error
// over the search directions of all of them.  With X, R, P the n-column
// blocks (n <= 8), per iteration
//     Q = A P,  alpha = (P^H Q)^-1 (R^H R),  X += P alpha,  R -= Q alpha,
//     beta = (R^H R)_old^-1 (R^H R)_new,  P = R + P beta,
// the n x n complex matrices in FP64 on the device (one thread, LU with
// partial pivoting).  Both Gram matrices are Hermitian in exact arithmetic;
// their upper triangles are summed and mirrored.  Every step runs in FP64.
// Block Krylov methods are the paper's route to fewer iterations for many
// right-hand sides (block BiCGStab on D in Sec. 3.1; this is the CG
// counterpart on the normal equations).
//
// Thread mapping: one thread per (site, component) of all n columns (grid.y =
// the 12 spin-colour components), so a thread holds one complex number of
// each column.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"
#include "handle.h"

namespace mfq {

constexpr int BCG_MAXN = 8;

struct BcgState {
  double g2r[BCG_MAXN * BCG_MAXN], g2i[BCG_MAXN * BCG_MAXN];  // R^H R, [i][j]
  double ar[BCG_MAXN * BCG_MAXN], ai[BCG_MAXN * BCG_MAXN];    // alpha, [j][i] multiplies column j into i
  double br[BCG_MAXN * BCG_MAXN], bi[BCG_MAXN * BCG_MAXN];    // beta, same convention
  double bnorm2[BCG_MAXN], rnorm2[BCG_MAXN];
  int done[BCG_MAXN];
  int breakdown;
  int count;      // iterations since the solve began (BETA steps)
  int converged;  // the count at which every column first met the tolerance, or -1
};

enum : int { BCG_INIT = 0, BCG_ALPHA = 1, BCG_BETA = 2 };

// upper-triangle index of (i, j), i <= j
__host__ __device__ constexpr int tri(int i, int j, int n) { return i * n - i * (i - 1) / 2 + (j - i); }

__device__ __forceinline__ void load1(const Field<double>& f, int rhs, int par, int comp, int s, cpx<double>& v) {
  const d2 q = f.data[f.cidx(rhs, par, comp, s)];
  v = {q.x, q.y};
}
__device__ __forceinline__ void store1(const Field<double>& f, int rhs, int par, int comp, int s,
                                       const cpx<double>& v) {
  d2 q;
  q.x = v.re;
  q.y = v.im;
  f.data[f.cidx(rhs, par, comp, s)] = q;
}

// One workgroup's partial of an upper-triangular Gram matrix (NE complex
// values): wave sums, then the 4 waves in a fixed order.
template <int NV>
__device__ __forceinline__ void bcg_block_partial(const double (&acc)[NV], double* part) {
  __shared__ double ws[4][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double v = wave_sum(acc[i]);
    if (lane == 0) ws[wv][i] = v;
  }
  __syncthreads();
  const long blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
  if (threadIdx.x < NV) {
    const int i = threadIdx.x;
    part[blk * NV + i] = ((ws[0][i] + ws[1][i]) + ws[2][i]) + ws[3][i];
  }
}

#define BCG_LANE                                          \
  const int q = blockIdx.x * blockDim.x + threadIdx.x;    \
  const int comp = blockIdx.y;                            \
  const bool valid = q < 2 * g.vh;                        \
  const int par = q >= g.vh ? 1 : 0;                      \
  const int s = valid ? q - par * g.vh : 0;

// Upper triangle of A^H B over all sites (A == B allowed).
template <int N>
__global__ __launch_bounds__(256) void bcg_gram_kernel(Geom g, Field<double> A, Field<double> B, double* part) {
  BCG_LANE
  constexpr int NV = N * (N + 1);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (valid) {
    cpx<double> a[N], b[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      load1(A, i, par, comp, s, a[i]);
      load1(B, i, par, comp, s, b[i]);
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) {
        const cpx<double> d = cjmul(a[i], b[j]);
        acc[2 * tri(i, j, N)] += d.re;
        acc[2 * tri(i, j, N) + 1] += d.im;
      }
  }
  bcg_block_partial<NV>(acc, part);
}

// X += P alpha, R -= Q alpha, and the upper triangle of the new R^H R.
template <int N>
__global__ __launch_bounds__(256) void bcg_xr_kernel(Geom g, Field<double> X, Field<double> R, Field<double> P,
                                                     Field<double> Q, const BcgState* st, double* part) {
  BCG_LANE
  constexpr int NV = N * (N + 1);
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (valid) {
    cpx<double> p[N], qq[N], r[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      load1(P, j, par, comp, s, p[j]);
      load1(Q, j, par, comp, s, qq[j]);
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      cpx<double> x;
      load1(X, i, par, comp, s, x);
      load1(R, i, par, comp, s, r[i]);
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const cpx<double> al = {st->ar[j * BCG_MAXN + i], st->ai[j * BCG_MAXN + i]};
        x = x + cmul(p[j], al);
        r[i] = r[i] - cmul(qq[j], al);
      }
      store1(X, i, par, comp, s, x);
      store1(R, i, par, comp, s, r[i]);
    }
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = i; j < N; ++j) {
        const cpx<double> d = cjmul(r[i], r[j]);
        acc[2 * tri(i, j, N)] += d.re;
        acc[2 * tri(i, j, N) + 1] += d.im;
      }
  }
  bcg_block_partial<NV>(acc, part);
}

// Pn = R + P beta (Pn and P distinct)
template <int N>
__global__ __launch_bounds__(256) void bcg_p_kernel(Geom g, Field<double> R, Field<double> P, Field<double> Pn,
                                                    const BcgState* st) {
  BCG_LANE
  if (!valid) return;
  cpx<double> p[N];
#pragma unroll
  for (int j = 0; j < N; ++j) load1(P, j, par, comp, s, p[j]);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    cpx<double> v;
    load1(R, i, par, comp, s, v);
#pragma unroll
    for (int j = 0; j < N; ++j) v = v + cmul(p[j], cpx<double>{st->br[j * BCG_MAXN + i], st->bi[j * BCG_MAXN + i]});
    store1(Pn, i, par, comp, s, v);
  }
}

// Solve M y = v (N x N complex) by Gaussian elimination with partial
// pivoting, everything in registers (compile-time indices: the pivot row is
// brought up by conditional swaps).  Returns false on a zero or non-finite
// pivot.
template <int N>
__device__ __forceinline__ bool solve_column(double (&mr)[N][N], double (&mi)[N][N], double (&vr)[N], double (&vi)[N]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < N; ++k) {
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const bool sw = fabs(mr[i][k]) + fabs(mi[i][k]) > fabs(mr[k][k]) + fabs(mi[k][k]);
#pragma unroll
      for (int c = k; c < N; ++c) {
        const double ar = mr[k][c], ai = mi[k][c], br = mr[i][c], bi = mi[i][c];
        mr[k][c] = sw ? br : ar;
        mi[k][c] = sw ? bi : ai;
        mr[i][c] = sw ? ar : br;
        mi[i][c] = sw ? ai : bi;
      }
      const double ar = vr[k], ai = vi[k], br = vr[i], bi = vi[i];
      vr[k] = sw ? br : ar;
      vi[k] = sw ? bi : ai;
      vr[i] = sw ? ar : br;
      vi[i] = sw ? ai : bi;
    }
    const double pr = mr[k][k], pi = mi[k][k];
    const double pd = pr * pr + pi * pi;
    ok = ok && pd > 0.0 && isfinite(pd);
    const double ipd = 1.0 / pd;  // 1 / M[k][k] = (pr - i pi) / pd
    const double qr = pr * ipd, qi = -pi * ipd;
    mr[k][k] = qr;  // keep the reciprocal pivot for the back substitution
    mi[k][k] = qi;
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const double xr = mr[i][k], xi = mi[i][k];
      const double fr = xr * qr - xi * qi, fi = xr * qi + xi * qr;  // M[i][k] / M[k][k]
#pragma unroll
      for (int c = k + 1; c < N; ++c) {
        mr[i][c] -= fr * mr[k][c] - fi * mi[k][c];
        mi[i][c] -= fr * mi[k][c] + fi * mr[k][c];
      }
      vr[i] -= fr * vr[k] - fi * vi[k];
      vi[i] -= fr * vi[k] + fi * vr[k];
    }
  }
#pragma unroll
  for (int k = N - 1; k >= 0; --k) {
    double sr = vr[k], si = vi[k];
#pragma unroll
    for (int l = k + 1; l < N; ++l) {
      sr -= mr[k][l] * vr[l] - mi[k][l] * vi[l];
      si -= mr[k][l] * vi[l] + mi[k][l] * vr[l];
    }
    const double qr = mr[k][k], qi = mi[k][k];  // reciprocal pivot
    vr[k] = sr * qr - si * qi;
    vi[k] = sr * qi + si * qr;
    ok = ok && isfinite(vr[k]) && isfinite(vi[k]);
  }
  return ok;
}

// Sum the Gram partials (fixed order: lanes over workgroups, then the wave
// sum) into a full Hermitian matrix G, then: INIT stores G as R^H R (and the
// convergence flags); ALPHA solves (P^H Q) alpha = R^H R; BETA solves
// (R^H R)_old beta = (R^H R)_new, keeps the new matrix and sets the
// convergence flags.  Thread j < N solves for column j.
template <int N>
__global__ __launch_bounds__(256) void bcg_small_kernel(const double* part, int nparts, int mode, double tol2,
                                                        BcgState* st) {
  __shared__ double gr[N][N], gi[N][N];
  __shared__ double ws[4][N * (N + 1)];
  __shared__ int bad;
  constexpr int NV = N * (N + 1);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) bad = 0;
  // every thread sums its share of the workgroup partials for all values
  // (independent loads in flight), then one fixed-order workgroup reduction
  double acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] += part[(long)b * NV + v];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const double x = wave_sum(acc[v]);
    if (lane == 0) ws[wv][v] = x;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int v = threadIdx.x;
    const double sum = ((ws[0][v] + ws[1][v]) + ws[2][v]) + ws[3][v];
    const int e = v / 2;
    int i = 0;
    while (e > tri(i, N - 1, N)) ++i;
    const int j = i + (e - tri(i, i, N));
    if (v % 2 == 0) {
      gr[i][j] = sum;
      gr[j][i] = sum;
    } else if (i != j) {
      gi[i][j] = sum;
      gi[j][i] = -sum;
    } else {
      gi[i][i] = 0.0;
    }
  }
  __syncthreads();
  BcgState& S = *st;
  const int t = threadIdx.x;
  if (mode != BCG_INIT && t < N) {
    double mr[N][N], mi[N][N], vr[N], vi[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
#pragma unroll
      for (int c = 0; c < N; ++c) {
        mr[i][c] = mode == BCG_ALPHA ? gr[i][c] : S.g2r[i * BCG_MAXN + c];
        mi[i][c] = mode == BCG_ALPHA ? gi[i][c] : S.g2i[i * BCG_MAXN + c];
      }
      vr[i] = mode == BCG_ALPHA ? S.g2r[i * BCG_MAXN + t] : gr[i][t];
      vi[i] = mode == BCG_ALPHA ? S.g2i[i * BCG_MAXN + t] : gi[i][t];
    }
    const bool ok = solve_column<N>(mr, mi, vr, vi);
    if (!ok) atomicOr(&bad, 1);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      if (mode == BCG_ALPHA) {
        S.ar[i * BCG_MAXN + t] = vr[i];
        S.ai[i * BCG_MAXN + t] = vi[i];
      } else {
        S.br[i * BCG_MAXN + t] = vr[i];
        S.bi[i * BCG_MAXN + t] = vi[i];
      }
    }
  }
  __syncthreads();
  if (t != 0) return;
  if (mode == BCG_ALPHA) {
    if (bad) {
      S.breakdown = 1;
      for (int k = 0; k < BCG_MAXN * BCG_MAXN; ++k) S.ar[k] = S.ai[k] = 0.0;
    }
    return;
  }
  if (mode == BCG_BETA) S.count += 1;
  for (int i = 0; i < N; ++i)
    for (int c = 0; c < N; ++c) {
      S.g2r[i * BCG_MAXN + c] = gr[i][c];
      S.g2i[i * BCG_MAXN + c] = gi[i][c];
    }
  bool all = true;
  for (int i = 0; i < N; ++i) {
    S.rnorm2[i] = gr[i][i];
    S.done[i] = S.rnorm2[i] <= tol2 * S.bnorm2[i];
    all = all && S.done[i];
  }
  if (mode == BCG_INIT) {
    S.breakdown = 0;
    return;
  }
  if (all && S.converged < 0) S.converged = S.count;
  if (bad) {
    for (int k = 0; k < BCG_MAXN * BCG_MAXN; ++k) S.br[k] = S.bi[k] = 0.0;
    // a singular (R^H R)_old with every column converged is the normal end
    if (!all) S.breakdown = 1;
  }
}

__global__ void bcg_bnorm_kernel(const double* part, int nparts, int n, BcgState* st) {
  // |b_i|^2 from the diagonal of the Gram partials of B (INIT runs next)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nv = n * (n + 1);
  for (int i = wv; i < n; i += 4) {
    const int v = 2 * tri(i, i, n);
    double sum = 0.0;
    for (int b = lane; b < nparts; b += 64) sum += part[(long)b * nv + v];
    sum = wave_sum(sum);
    if (lane == 0) st->bnorm2[i] = sum;
  }
  if (threadIdx.x == 0) {
    st->count = 0;
    st->converged = -1;
  }
}

// out = a - b, or a += b (sub = 0), over all n fields
__global__ __launch_bounds__(256) void bcg_combine_kernel(Geom g, Field<double> a, Field<double> b,
                                                          Field<double> out, int n, int sub) {
  BCG_LANE
  if (!valid) return;
  for (int i = 0; i < n; ++i) {
    cpx<double> x, y;
    load1(a, i, par, comp, s, x);
    load1(b, i, par, comp, s, y);
    store1(out, i, par, comp, s, sub ? x - y : x + y);
  }
}

#define BCG_N_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
static_assert(BCG_MAXN == 8, "one kernel instance per block size 1..BCG_MAXN");

hipError_t bcg_small(int n, hipStream_t st, const double* part, int nparts, int mode, double tol2, BcgState* S) {
  switch (n) {
#define BCG_S(N)                                                                                       \
  case N:                                                                                              \
    hipLaunchKernelGGL((bcg_small_kernel<N>), dim3(1), dim3(256), 0, st, part, nparts, mode, tol2, S); \
    break;
    BCG_N_CASES(BCG_S)
#undef BCG_S
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t bcg_gram(int n, dim3 grid, hipStream_t st, const Geom& g, Field<double> A, Field<double> B, double* part) {
  switch (n) {
#define BCG_G(N)                                                                            \
  case N:                                                                                   \
    hipLaunchKernelGGL((bcg_gram_kernel<N>), grid, dim3(256), 0, st, g, A, B, part);      \
    break;
    BCG_N_CASES(BCG_G)
#undef BCG_G
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t bcg_xr(int n, dim3 grid, hipStream_t st, const Geom& g, Field<double> X, Field<double> R, Field<double> P,
                  Field<double> Q, const BcgState* S, double* part) {
  switch (n) {
#define BCG_X(N)                                                                                \
  case N:                                                                                       \
    hipLaunchKernelGGL((bcg_xr_kernel<N>), grid, dim3(256), 0, st, g, X, R, P, Q, S, part);   \
    break;
    BCG_N_CASES(BCG_X)
#undef BCG_X
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t bcg_p(int n, dim3 grid, hipStream_t st, const Geom& g, Field<double> R, Field<double> P, Field<double> Pn,
                 const BcgState* S) {
  switch (n) {
#define BCG_P(N)                                                                         \
  case N:                                                                                \
    hipLaunchKernelGGL((bcg_p_kernel<N>), grid, dim3(256), 0, st, g, R, P, Pn, S);     \
    break;
    BCG_N_CASES(BCG_P)
#undef BCG_P
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Block CG on D^+D x64 = b64 (packed FP64), n <= BCG_MAXN RHS.
int run_block_cg(mfq_handle* h, int n, const mfq_solve_params* P, hipStream_t st, mfq_solve_stats* stats) {
  const Geom& g = h->g;
  Workspace& w = h->ws;
  if (n > BCG_MAXN) return fail(MFQ_ERR_ARG, "block CG takes at most 8 right-hand sides");
  if (P->prec != MFQ_PREC_FP64) return fail(MFQ_ERR_ARG, "block CG runs in FP64 (prec must be MFQ_PREC_FP64)");
  Shape sh;
  if (int rc = fp64_hop_shape(h, n, st, &sh)) return rc;
  OwnedField<double> fr, fp, fq, fpn, fxs, fbs;
  DevBuf stb, partb;
  auto cleanup = [&]() {
    for (auto* f : {&fr, &fp, &fq, &fpn, &fxs, &fbs}) f->free_all();
    release(stb);
    release(partb);
  };
  const int nblk = (2 * g.vh + 255) / 256;
  const dim3 grid(nblk, 12);
  const int nparts = nblk * 12;
  if (fr.alloc(g, n) || fp.alloc(g, n) || fq.alloc(g, n) || fpn.alloc(g, n) || ensure(stb, sizeof(BcgState)) ||
      ensure(partb, sizeof(double) * (size_t)nparts * n * (n + 1))) {
    cleanup();
    return fail(MFQ_ERR_NOMEM, "block CG workspace");
  }
  BcgState* S = (BcgState*)stb.ptr;
  double* part = (double*)partb.ptr;
  Field<double> R = fr.view(g), Pf = fp.view(g), Q = fq.view(g), Pn = fpn.view(g);
  Field<double> b64 = w.b64.view(g), x64 = w.x64.view(g), r64 = w.r64.view(g), t64 = w.t64.view(g);
  const size_t fbytes = field_chunks<double>(g, n) * sizeof(d2);
  const double tol2 = P->tol * P->tol;
  HopArgs<double, double> a = hop_args<double, double>(h, links_d(h), n);
  a.coef = -h->lat.kappa;
  a.par = 2;
  auto apply_a = [&](Field<double> in, Field<double> out) -> int {
    a.in = a.self = in;
    a.out = t64;
    a.dagger = 0;
    HIPCHK(launch_hop<double, double>(EPI_D, a, sh, st));
    a.in = a.self = t64;
    a.out = out;
    a.dagger = 1;
    HIPCHK(launch_hop<double, double>(EPI_D, a, sh, st));
    return MFQ_OK;
  };
  auto combine = [&](Field<double> x, Field<double> y, Field<double> out, int sub) -> int {
    hipLaunchKernelGGL(bcg_combine_kernel, grid, dim3(256), 0, st, g, x, y, out, n, sub);
    return hipGetLastError() == hipSuccess ? MFQ_OK : fail(MFQ_ERR_HIP, "bcg_combine");
  };
  auto small = [&](int mode) -> int {
    return bcg_small(n, st, part, nparts, mode, tol2, S) == hipSuccess ? MFQ_OK : fail(MFQ_ERR_HIP, "bcg_small");
  };
  BcgState host;
  // r64 = b - A x and its norms into host (rnorm2, done)
  auto true_residual = [&]() -> int {
    if (int rc = apply_a(x64, Q)) return rc;
    if (int rc = combine(b64, Q, r64, 1)) return rc;
    HIPCHK(bcg_gram(n, grid, st, g, r64, r64, part));
    if (int rc = small(BCG_INIT)) return rc;
    HIPCHK(hipMemcpyAsync(&host, S, sizeof(BcgState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MFQ_OK;
  };
  // (re)start from x64: R = b - A x (or b for x = 0), P = R, R^H R
  auto restart = [&](bool zero_x) -> int {
    if (zero_x) {
      HIPCHK(hipMemsetAsync(x64.data, 0, fbytes, st));
      HIPCHK(hipMemcpyAsync(R.data, b64.data, fbytes, hipMemcpyDeviceToDevice, st));
    } else {
      if (int rc = apply_a(x64, Q)) return rc;
      if (int rc = combine(b64, Q, R, 1)) return rc;
    }
    HIPCHK(hipMemcpyAsync(Pf.data, R.data, fbytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(bcg_gram(n, grid, st, g, R, R, part));
    return small(BCG_INIT);
  };
  int rc;
  HIPCHK(hipMemsetAsync(S, 0, sizeof(BcgState), st));
  HIPCHK(bcg_gram(n, grid, st, g, b64, b64, part));
  hipLaunchKernelGGL(bcg_bnorm_kernel, dim3(1), dim3(256), 0, st, part, nparts, n, S);
  HIPCHK(hipGetLastError());
  if ((rc = restart(true))) return cleanup(), rc;
  // one iteration on stream s with search directions Pa, new ones into Pb
  auto iteration = [&](hipStream_t s, Field<double> Pa, Field<double> Pb) -> int {
    a.in = a.self = Pa;
    a.out = t64;
    a.dagger = 0;
    HIPCHK(launch_hop<double, double>(EPI_D, a, sh, s));
    a.in = a.self = t64;
    a.out = Q;
    a.dagger = 1;
    HIPCHK(launch_hop<double, double>(EPI_D, a, sh, s));
    HIPCHK(bcg_gram(n, grid, s, g, Pa, Q, part));
    HIPCHK(bcg_small(n, s, part, nparts, BCG_ALPHA, tol2, S));
    HIPCHK(bcg_xr(n, grid, s, g, x64, R, Pa, Q, S, part));
    HIPCHK(bcg_small(n, s, part, nparts, BCG_BETA, tol2, S));
    HIPCHK(bcg_p(n, grid, s, g, R, Pa, Pb, S));
    return MFQ_OK;
  };
  // two iterations (P -> Pn -> P) captured once and replayed between polls
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  auto drop_graph = [&]() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
  };
  auto fail_all = [&](int code) {
    drop_graph();
    cleanup();
    return code;
  };
  const int every = P->check_every > 0 ? P->check_every + (P->check_every & 1) : 8;
  int iters = 0, restarts = 0;
  bool breakdown = false;
  for (;;) {
    // iterate until the recursive residuals claim convergence
    while (iters < P->max_iter) {
      const int k = every < P->max_iter - iters ? every : P->max_iter - iters;
      if (P->use_graph && k >= 2) {
        if (!gexec) {
          HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
          int rc2 = iteration(h->cap_stream, Pf, Pn);
          if (rc2 == MFQ_OK) rc2 = iteration(h->cap_stream, Pn, Pf);
          hipError_t ec = hipStreamEndCapture(h->cap_stream, &graph);
          if (rc2 != MFQ_OK) return fail_all(rc2);
          if (ec != hipSuccess) return fail_all(fail_hip(ec, "block CG capture"));
          if ((ec = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0)) != hipSuccess)
            return fail_all(fail_hip(ec, "block CG graph"));
        }
        for (int it = 0; it + 1 < k; it += 2) {
          hipError_t ec = hipGraphLaunch(gexec, st);
          if (ec != hipSuccess) return fail_all(fail_hip(ec, "block CG graph launch"));
        }
        iters += k & ~1;
        if (k & 1) {  // the last iteration before max_iter
          if ((rc = iteration(st, Pf, Pn))) return fail_all(rc);
          std::swap(Pf, Pn);
          iters += 1;
        }
      } else {
        for (int it = 0; it < k; ++it) {
          if ((rc = iteration(st, Pf, Pn))) return fail_all(rc);
          std::swap(Pf, Pn);
        }
        iters += k;
      }
      if (hipError_t ec = hipMemcpyAsync(&host, S, sizeof(BcgState), hipMemcpyDeviceToHost, st); ec != hipSuccess) return fail_all(fail_hip(ec, "block CG"));
      if (hipError_t ec = hipStreamSynchronize(st); ec != hipSuccess) return fail_all(fail_hip(ec, "block CG"));
      bool all_done = true;
      for (int i = 0; i < n; ++i) all_done = all_done && host.done[i];
      if (host.breakdown) breakdown = true;
      if (all_done || breakdown) break;
    }
    if ((rc = true_residual())) return fail_all(rc);
    bool ok = true;
    for (int i = 0; i < n; ++i) ok = ok && host.done[i];
    if (ok || breakdown || iters >= P->max_iter || restarts >= 3) break;
    // the recursion drifted from the true residual: restart from x
    ++restarts;
    if ((rc = restart(false))) return fail_all(rc);
  }
  bool all_ok = true;
  for (int i = 0; i < n; ++i) all_ok = all_ok && host.done[i];
  int status = all_ok ? MFQ_OK : MFQ_NOT_CONVERGED;
  int cg_iters = 0;
  if (breakdown && !all_ok) {
    // batched CG on A e = r (r64 holds the true residual), then x += e; the
    // residual system's tolerance keeps |b - A x| <= tol |b| for every RHS
    if (fxs.alloc(g, n) || fbs.alloc(g, n)) return fail_all(fail(MFQ_ERR_NOMEM, "block CG fallback"));
    double ratio = 1.0;
    for (int i = 0; i < n; ++i)
      if (host.rnorm2[i] > 0 && host.bnorm2[i] > 0 && std::isfinite(host.rnorm2[i]))
        ratio = fmin(ratio, sqrt(host.bnorm2[i] / host.rnorm2[i]));
    if (hipError_t ec = hipMemcpyAsync(fxs.view(g).data, x64.data, fbytes, hipMemcpyDeviceToDevice, st); ec != hipSuccess) return fail_all(fail_hip(ec, "block CG"));
    if (hipError_t ec = hipMemcpyAsync(fbs.view(g).data, b64.data, fbytes, hipMemcpyDeviceToDevice, st); ec != hipSuccess) return fail_all(fail_hip(ec, "block CG"));
    if (hipError_t ec = hipMemcpyAsync(b64.data, r64.data, fbytes, hipMemcpyDeviceToDevice, st); ec != hipSuccess) return fail_all(fail_hip(ec, "block CG"));
    mfq_solve_params Q2 = *P;
    Q2.precond = MFQ_PC_NONE;
    Q2.tol = fmax(fmin(P->tol * ratio, 0.5), 1e-15);
    std::vector<mfq_solve_stats> cst(n);
    rc = solve_packed(h, n, &Q2, st, cst.data());
    if (rc < 0) return fail_all(rc);
    for (int i = 0; i < n; ++i) cg_iters = cg_iters > cst[i].iters ? cg_iters : cst[i].iters;
    if ((rc = combine(x64, fxs.view(g), x64, 0))) return fail_all(rc);
    if (hipError_t ec = hipMemcpyAsync(b64.data, fbs.view(g).data, fbytes, hipMemcpyDeviceToDevice, st); ec != hipSuccess) return fail_all(fail_hip(ec, "block CG"));
    if ((rc = true_residual())) return fail_all(rc);
    all_ok = true;
    for (int i = 0; i < n; ++i) all_ok = all_ok && host.done[i];
    status = all_ok ? MFQ_FELL_BACK : MFQ_NOT_CONVERGED;
  }
  drop_graph();
  cleanup();
  // iterations until every column met the tolerance (polls come every few
  // iterations, so the loop may have run a few more), plus any CG hand-over
  const int it_conv = host.converged >= 0 && host.converged <= iters ? host.converged : iters;
  for (int i = 0; stats && i < n; ++i) {
    stats[i].iters = it_conv + cg_iters;
    stats[i].reliable_updates = restarts;
    stats[i].true_rel_resid = host.bnorm2[i] > 0 ? sqrt(host.rnorm2[i] / host.bnorm2[i]) : 0.0;
    stats[i].status = host.done[i] ? (status == MFQ_FELL_BACK ? MFQ_FELL_BACK : MFQ_OK) : MFQ_NOT_CONVERGED;
  }
  return status;
}

}  // namespace mfq
