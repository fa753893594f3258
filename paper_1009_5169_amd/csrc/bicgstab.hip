// The paper's solver family on the even/odd-preconditioned Wilson operator
// D^ = 1 - kappa^2 H_eo H_oe (Sec. 3.1: the blocked equations solved by
// BiCGStab, Global BiCGStab or Block BiCGStab; Sec. 3.2: a double-precision
// outer iteration whose preconditioner is a single-precision inner solve per
// right-hand side).  For the n <= 8 columns of one block:
//
//   V = A P^,  alpha from (R~^H V) alpha = R~^H R,  S = R - V alpha,
//   T = A S^,  omega = <T, S> / <T, T>,  X += P^ alpha + omega S^,
//   R = S - omega T,  beta from (R~^H V) beta = -R~^H T,
//   P = R + (P - omega V) beta,
//
// with R~ the residual block at the (re)start, P^ = K^-1 P and S^ = K^-1 S
// (the identity without preconditioner).  The three forms differ only in
// these small systems:
//   plain   every column its own BiCGStab: the diagonals (alpha_i =
//           (r~_i, r_i) / (r~_i, v_i), omega_i = (t_i, s_i) / (t_i, t_i),
//           beta_i = -(r~_i, t_i) / (r~_i, v_i)); a converged column freezes;
//   global  the same with Frobenius products summed over the columns, one
//           alpha, omega, beta for the block;
//   block   alpha and beta n x n (LU with partial pivoting), omega the
//           Frobenius ratio.
// (The beta forms equal van der Vorst's (rho'/rho)(alpha/omega), since
// R~^H S = 0 after the alpha step.)
//
// Vectors live on the even sites (the Schur system); the odd half of V and
// T holds the intermediate H_oe of each operator application.  Thread
// mapping: one thread per (even site, 16-byte chunk) holding that chunk of
// all n columns, like the block CG kernels.
#include <cmath>
#include <cstddef>
#include <cstring>
#include <vector>

#include "handle.h"
#include "hop_impl.h"
#include "internal.h"

namespace mfq {

constexpr int BI_MAXN = 8;
enum : int { BI_PLAIN = 0, BI_GLOBAL = 1, BI_BLOCK = 2 };
enum : int { BS_INIT = 0, BS_ALPHA = 1, BS_OMEGA = 2, BS_RES = 3 };

struct BiState {
  double g0r[BI_MAXN * BI_MAXN], g0i[BI_MAXN * BI_MAXN];  // R~^H R, [i][j] = r~_i^H r_j
  double g1r[BI_MAXN * BI_MAXN], g1i[BI_MAXN * BI_MAXN];  // R~^H V
  double ar[BI_MAXN * BI_MAXN], ai[BI_MAXN * BI_MAXN];    // alpha [j][i]: column j into column i
  double br[BI_MAXN * BI_MAXN], bi[BI_MAXN * BI_MAXN];    // beta, same convention
  double wr[BI_MAXN], wi[BI_MAXN];                        // omega per column
  double bnorm2[BI_MAXN], rnorm2[BI_MAXN];
  int done[BI_MAXN];
  int frozen[BI_MAXN];  // plain form: the column has converged and stopped
  int breakdown;
  int count;      // iterations since the solve began
  int converged;  // the count at which every column first met the tolerance, or -1
};

// ---------------------------------------------------------------- chunk I/O
template <typename S>
struct Chunk;
template <>
struct Chunk<double> {
  static constexpr int C = 1;  // complex values per 16-byte chunk
  __device__ static void load(const Field<double>& f, int r, int c, int s, cpx<double> v[1]) {
    const d2 q = f.data[f.cidx(r, 0, c, s)];
    v[0] = {q.x, q.y};
  }
  __device__ static void store(const Field<double>& f, int r, int c, int s, const cpx<double> v[1]) {
    d2 q;
    q.x = v[0].re;
    q.y = v[0].im;
    f.data[f.cidx(r, 0, c, s)] = q;
  }
};
template <>
struct Chunk<float> {
  static constexpr int C = 2;
  __device__ static void load(const Field<float>& f, int r, int c, int s, cpx<float> v[2]) {
    const f4 q = f.data[f.cidx(r, 0, c, s)];
    v[0] = {q.x, q.y};
    v[1] = {q.z, q.w};
  }
  __device__ static void store(const Field<float>& f, int r, int c, int s, const cpx<float> v[2]) {
    f4 q;
    q.x = v[0].re;
    q.y = v[0].im;
    q.z = v[1].re;
    q.w = v[1].im;
    f.data[f.cidx(r, 0, c, s)] = q;
  }
};

template <int NV>
__device__ __forceinline__ void bi_block_partial(const double (&acc)[NV], double* part) {
  __shared__ double ws[4][NV];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const double v = wave_sum(acc[i]);
    if (lane == 0) ws[wv][i] = v;
  }
  __syncthreads();
  const long blk = (long)blockIdx.y * gridDim.x + blockIdx.x;
  for (int i = threadIdx.x; i < NV; i += blockDim.x) part[blk * NV + i] = ((ws[0][i] + ws[1][i]) + ws[2][i]) + ws[3][i];
}

#define BI_LANE                                       \
  const int s = blockIdx.x * blockDim.x + threadIdx.x; \
  const int c = blockIdx.y;                            \
  const bool valid = s < g.vh;

// Gram values over the even sites.  Layouts of one workgroup's partial:
//   GRAM_FULL  (A, B): 2 N^2 values, A^H B row-major [i][j] (re, im)
//   GRAM_TS    (T, S, R~): diag(T^H S) (2N), diag(T^H T) (N), R~^H T (2 N^2)
enum : int { GRAM_FULL = 0, GRAM_TS = 1 };
template <int N, int MODE>
constexpr int gram_nv() {
  return MODE == GRAM_FULL ? 2 * N * N : 3 * N + 2 * N * N;
}

template <int N, int MODE, typename S>
__global__ __launch_bounds__(256) void bi_gram_kernel(Geom g, Field<S> A, Field<S> B, Field<S> Rt, double* part) {
  BI_LANE
  constexpr int NV = gram_nv<N, MODE>();
  constexpr int C = Chunk<S>::C;
  using T = typename Compute<S>::T;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (valid) {
    cpx<T> a[N][C], b[N][C];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Chunk<S>::load(A, i, c, s, a[i]);
      Chunk<S>::load(B, i, c, s, b[i]);
    }
    if constexpr (MODE == GRAM_FULL) {
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
          for (int q = 0; q < C; ++q) {
            const cpx<T> d = cjmul(a[i][q], b[j][q]);
            acc[2 * (i * N + j)] += (double)d.re;
            acc[2 * (i * N + j) + 1] += (double)d.im;
          }
    } else {  // A = T, B = S
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int q = 0; q < C; ++q) {
          const cpx<T> d = cjmul(a[i][q], b[i][q]);
          acc[2 * i] += (double)d.re;
          acc[2 * i + 1] += (double)d.im;
          acc[2 * N + i] += (double)norm2(a[i][q]);
        }
      cpx<T> rt[N][C];
#pragma unroll
      for (int i = 0; i < N; ++i) Chunk<S>::load(Rt, i, c, s, rt[i]);
#pragma unroll
      for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
          for (int q = 0; q < C; ++q) {
            const cpx<T> d = cjmul(rt[i][q], a[j][q]);
            acc[3 * N + 2 * (i * N + j)] += (double)d.re;
            acc[3 * N + 2 * (i * N + j) + 1] += (double)d.im;
          }
    }
  }
  bi_block_partial<NV>(acc, part);
}

// S = R - V alpha
template <int N, typename S>
__global__ __launch_bounds__(256) void bi_s_kernel(Geom g, Field<S> R, Field<S> V, Field<S> Sf, const BiState* st) {
  BI_LANE
  if (!valid) return;
  constexpr int C = Chunk<S>::C;
  using T = typename Compute<S>::T;
  cpx<T> v[N][C];
#pragma unroll
  for (int j = 0; j < N; ++j) Chunk<S>::load(V, j, c, s, v[j]);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    cpx<T> r[C];
    Chunk<S>::load(R, i, c, s, r);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const cpx<T> al = {(T)st->ar[j * BI_MAXN + i], (T)st->ai[j * BI_MAXN + i]};
#pragma unroll
      for (int q = 0; q < C; ++q) r[q] = r[q] - cmul(v[j][q], al);
    }
    Chunk<S>::store(Sf, i, c, s, r);
  }
}

// X += P^ alpha + omega S^;  R = S - omega T;  partials of R~^H R (2 N^2) and
// diag(R^H R) (N)
template <int N, typename S>
__global__ __launch_bounds__(256) void bi_xr_kernel(Geom g, Field<S> X, Field<S> R, Field<S> Ph, Field<S> Sf,
                                                    Field<S> Sh, Field<S> Tf, Field<S> Rt, const BiState* st,
                                                    double* part) {
  BI_LANE
  constexpr int C = Chunk<S>::C;
  constexpr int NV = 2 * N * N + N;
  using T = typename Compute<S>::T;
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  if (valid) {
    cpx<T> ph[N][C], r[N][C];
#pragma unroll
    for (int j = 0; j < N; ++j) Chunk<S>::load(Ph, j, c, s, ph[j]);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      cpx<T> x[C], sv[C], sh[C], t[C];
      Chunk<S>::load(X, i, c, s, x);
      Chunk<S>::load(Sf, i, c, s, sv);
      Chunk<S>::load(Sh, i, c, s, sh);
      Chunk<S>::load(Tf, i, c, s, t);
      const cpx<T> om = {(T)st->wr[i], (T)st->wi[i]};
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const cpx<T> al = {(T)st->ar[j * BI_MAXN + i], (T)st->ai[j * BI_MAXN + i]};
#pragma unroll
        for (int q = 0; q < C; ++q) x[q] = x[q] + cmul(ph[j][q], al);
      }
#pragma unroll
      for (int q = 0; q < C; ++q) {
        x[q] = x[q] + cmul(om, sh[q]);
        r[i][q] = sv[q] - cmul(om, t[q]);
        acc[2 * N * N + i] += (double)norm2(r[i][q]);
      }
      Chunk<S>::store(X, i, c, s, x);
      Chunk<S>::store(R, i, c, s, r[i]);
    }
    cpx<T> rt[N][C];
#pragma unroll
    for (int i = 0; i < N; ++i) Chunk<S>::load(Rt, i, c, s, rt[i]);
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
      for (int j = 0; j < N; ++j)
#pragma unroll
        for (int q = 0; q < C; ++q) {
          const cpx<T> d = cjmul(rt[i][q], r[j][q]);
          acc[2 * (i * N + j)] += (double)d.re;
          acc[2 * (i * N + j) + 1] += (double)d.im;
        }
  }
  bi_block_partial<NV>(acc, part);
}

// P = R + (P - omega V) beta  (in place: every column of the chunk is read first)
template <int N, typename S>
__global__ __launch_bounds__(256) void bi_p_kernel(Geom g, Field<S> R, Field<S> P, Field<S> V, const BiState* st) {
  BI_LANE
  if (!valid) return;
  constexpr int C = Chunk<S>::C;
  using T = typename Compute<S>::T;
  cpx<T> w[N][C];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    cpx<T> p[C], v[C];
    Chunk<S>::load(P, j, c, s, p);
    Chunk<S>::load(V, j, c, s, v);
    const cpx<T> om = {(T)st->wr[j], (T)st->wi[j]};
#pragma unroll
    for (int q = 0; q < C; ++q) w[j][q] = p[q] - cmul(om, v[q]);
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    cpx<T> r[C];
    Chunk<S>::load(R, i, c, s, r);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const cpx<T> be = {(T)st->br[j * BI_MAXN + i], (T)st->bi[j * BI_MAXN + i]};
#pragma unroll
      for (int q = 0; q < C; ++q) r[q] = r[q] + cmul(w[j][q], be);
    }
    Chunk<S>::store(P, i, c, s, r);
  }
}

// out = a - b (sub) or out = a (copy) over all n columns
template <typename S>
__global__ __launch_bounds__(256) void bi_combine_kernel(Geom g, Field<S> a, Field<S> b, Field<S> out, int n, int sub) {
  BI_LANE
  if (!valid) return;
  constexpr int C = Chunk<S>::C;
  using T = typename Compute<S>::T;
  for (int i = 0; i < n; ++i) {
    cpx<T> x[C], y[C];
    Chunk<S>::load(a, i, c, s, x);
    if (sub) {
      Chunk<S>::load(b, i, c, s, y);
#pragma unroll
      for (int q = 0; q < C; ++q) x[q] = x[q] - y[q];
    }
    Chunk<S>::store(out, i, c, s, x);
  }
}

// Solve M y = v (N x N complex) by Gaussian elimination with partial
// pivoting in registers; false on a zero or non-finite pivot.
template <int N>
__device__ __forceinline__ bool bi_solve(double (&mr)[N][N], double (&mi)[N][N], double (&vr)[N], double (&vi)[N]) {
  bool ok = true;
#pragma unroll
  for (int k = 0; k < N; ++k) {
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const bool sw = fabs(mr[i][k]) + fabs(mi[i][k]) > fabs(mr[k][k]) + fabs(mi[k][k]);
#pragma unroll
      for (int cc = k; cc < N; ++cc) {
        const double ar = mr[k][cc], ai = mi[k][cc], br = mr[i][cc], bi = mi[i][cc];
        mr[k][cc] = sw ? br : ar;
        mi[k][cc] = sw ? bi : ai;
        mr[i][cc] = sw ? ar : br;
        mi[i][cc] = sw ? ai : bi;
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
    const double qr = pr / pd, qi = -pi / pd;
    mr[k][k] = qr;
    mi[k][k] = qi;
#pragma unroll
    for (int i = k + 1; i < N; ++i) {
      const double fr = mr[i][k] * qr - mi[i][k] * qi, fi = mr[i][k] * qi + mi[i][k] * qr;
#pragma unroll
      for (int cc = k + 1; cc < N; ++cc) {
        mr[i][cc] -= fr * mr[k][cc] - fi * mi[k][cc];
        mi[i][cc] -= fr * mi[k][cc] + fi * mr[k][cc];
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
    vr[k] = sr * mr[k][k] - si * mi[k][k];
    vi[k] = sr * mi[k][k] + si * mr[k][k];
    ok = ok && isfinite(vr[k]) && isfinite(vi[k]);
  }
  return ok;
}

// complex a / b
__device__ __forceinline__ void cdiv(double ar, double ai, double br, double bi, double& qr, double& qi) {
  const double d = br * br + bi * bi;
  qr = (ar * br + ai * bi) / d;
  qi = (ai * br - ar * bi) / d;
}

// Sum the partials in a fixed order (every thread strides over the
// workgroups for all values, then one workgroup reduction), then update the
// state for `mode` (one thread; block solves one column per thread).
template <int N>
__global__ __launch_bounds__(256) void bi_small_kernel(const double* part, int nparts, int mode, int kind,
                                                       double tol2, BiState* st) {
  constexpr int NVMAX = 3 * N + 2 * N * N;
  const int nv = mode == BS_ALPHA ? 2 * N * N : (mode == BS_OMEGA ? 3 * N + 2 * N * N : 2 * N * N + N);
  __shared__ double ws[4][NVMAX];
  __shared__ double sum[NVMAX];
  __shared__ int bad;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) bad = 0;
  double acc[NVMAX];
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) acc[v] = 0.0;
  for (int b = threadIdx.x; b < nparts; b += blockDim.x)
    for (int v = 0; v < nv; ++v) acc[v] += part[(long)b * nv + v];
#pragma unroll
  for (int v = 0; v < NVMAX; ++v) {
    const double x = wave_sum(acc[v]);
    if (lane == 0) ws[wv][v] = x;
  }
  __syncthreads();
  for (int v = threadIdx.x; v < nv; v += blockDim.x) sum[v] = ((ws[0][v] + ws[1][v]) + ws[2][v]) + ws[3][v];
  __syncthreads();
  BiState& S = *st;
  const int t = threadIdx.x;
  if (mode == BS_ALPHA) {
    // sum = R~^H V;  alpha
    if (t == 0) {
      for (int i = 0; i < N; ++i)
        for (int j = 0; j < N; ++j) {
          S.g1r[i * BI_MAXN + j] = sum[2 * (i * N + j)];
          S.g1i[i * BI_MAXN + j] = sum[2 * (i * N + j) + 1];
          S.ar[i * BI_MAXN + j] = S.ai[i * BI_MAXN + j] = 0.0;
        }
      if (kind == BI_PLAIN) {
        for (int i = 0; i < N; ++i) {
          if (S.frozen[i]) continue;
          double qr, qi;
          const double dr = S.g1r[i * BI_MAXN + i], di = S.g1i[i * BI_MAXN + i];
          if (dr * dr + di * di > 0.0) {
            cdiv(S.g0r[i * BI_MAXN + i], S.g0i[i * BI_MAXN + i], dr, di, qr, qi);
            S.ar[i * BI_MAXN + i] = qr;
            S.ai[i * BI_MAXN + i] = qi;
          } else {
            bad = 1;
          }
        }
      } else if (kind == BI_GLOBAL) {
        double nr = 0, ni = 0, dr = 0, di = 0;
        for (int i = 0; i < N; ++i) {
          nr += S.g0r[i * BI_MAXN + i];
          ni += S.g0i[i * BI_MAXN + i];
          dr += S.g1r[i * BI_MAXN + i];
          di += S.g1i[i * BI_MAXN + i];
        }
        if (dr * dr + di * di > 0.0) {
          double qr, qi;
          cdiv(nr, ni, dr, di, qr, qi);
          for (int i = 0; i < N; ++i) {
            S.ar[i * BI_MAXN + i] = qr;
            S.ai[i * BI_MAXN + i] = qi;
          }
        } else {
          bad = 1;
        }
      }
    }
    __syncthreads();
    if (kind == BI_BLOCK && t < N) {
      // column t of alpha: (R~^H V) a = (R~^H R)[:, t]
      double mr[N][N], mi[N][N], vr[N], vi[N];
#pragma unroll
      for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int cc = 0; cc < N; ++cc) {
          mr[i][cc] = sum[2 * (i * N + cc)];
          mi[i][cc] = sum[2 * (i * N + cc) + 1];
        }
        vr[i] = S.g0r[i * BI_MAXN + t];
        vi[i] = S.g0i[i * BI_MAXN + t];
      }
      if (!bi_solve<N>(mr, mi, vr, vi)) atomicOr(&bad, 1);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        S.ar[i * BI_MAXN + t] = vr[i];
        S.ai[i * BI_MAXN + t] = vi[i];
      }
    }
    __syncthreads();
    if (t == 0 && bad) {
      S.breakdown = 1;
      for (int k = 0; k < BI_MAXN * BI_MAXN; ++k) S.ar[k] = S.ai[k] = 0.0;
    }
    return;
  }
  if (mode == BS_OMEGA) {
    // sum = diag(T^H S) (2N), diag(T^H T) (N), R~^H T (2 N^2): omega, then beta
    const double* c3 = sum + 3 * N;
    if (t == 0) {
      for (int k = 0; k < BI_MAXN * BI_MAXN; ++k) S.br[k] = S.bi[k] = 0.0;
      double nr = 0, ni = 0, dd = 0;
      for (int i = 0; i < N; ++i) {
        S.wr[i] = S.wi[i] = 0.0;
        if (kind == BI_PLAIN) {
          if (S.frozen[i]) continue;
          if (sum[2 * N + i] > 0.0) {
            S.wr[i] = sum[2 * i] / sum[2 * N + i];
            S.wi[i] = sum[2 * i + 1] / sum[2 * N + i];
          } else {
            bad = 1;
          }
        } else {
          nr += sum[2 * i];
          ni += sum[2 * i + 1];
          dd += sum[2 * N + i];
        }
      }
      if (kind != BI_PLAIN) {
        if (dd > 0.0) {
          for (int i = 0; i < N; ++i) {
            S.wr[i] = nr / dd;
            S.wi[i] = ni / dd;
          }
        } else {
          bad = 1;
        }
      }
      if (kind == BI_PLAIN) {
        for (int i = 0; i < N; ++i) {
          if (S.frozen[i]) continue;
          const double dr = S.g1r[i * BI_MAXN + i], di = S.g1i[i * BI_MAXN + i];
          double qr, qi;
          cdiv(-c3[2 * (i * N + i)], -c3[2 * (i * N + i) + 1], dr, di, qr, qi);
          S.br[i * BI_MAXN + i] = qr;
          S.bi[i * BI_MAXN + i] = qi;
        }
      } else if (kind == BI_GLOBAL) {
        double tr = 0, ti = 0, dr = 0, di = 0;
        for (int i = 0; i < N; ++i) {
          tr += c3[2 * (i * N + i)];
          ti += c3[2 * (i * N + i) + 1];
          dr += S.g1r[i * BI_MAXN + i];
          di += S.g1i[i * BI_MAXN + i];
        }
        double qr, qi;
        cdiv(-tr, -ti, dr, di, qr, qi);
        for (int i = 0; i < N; ++i) {
          S.br[i * BI_MAXN + i] = qr;
          S.bi[i * BI_MAXN + i] = qi;
        }
      }
    }
    __syncthreads();
    if (kind == BI_BLOCK && t < N) {
      double mr[N][N], mi[N][N], vr[N], vi[N];
#pragma unroll
      for (int i = 0; i < N; ++i) {
#pragma unroll
        for (int cc = 0; cc < N; ++cc) {
          mr[i][cc] = S.g1r[i * BI_MAXN + cc];
          mi[i][cc] = S.g1i[i * BI_MAXN + cc];
        }
        vr[i] = -c3[2 * (i * N + t)];
        vi[i] = -c3[2 * (i * N + t) + 1];
      }
      if (!bi_solve<N>(mr, mi, vr, vi)) atomicOr(&bad, 1);
#pragma unroll
      for (int i = 0; i < N; ++i) {
        S.br[i * BI_MAXN + t] = vr[i];
        S.bi[i * BI_MAXN + t] = vi[i];
      }
    }
    __syncthreads();
    if (t == 0 && bad) {
      S.breakdown = 1;
      for (int k = 0; k < BI_MAXN; ++k) S.wr[k] = S.wi[k] = 0.0;
    }
    return;
  }
  // BS_INIT / BS_RES: sum = R~^H R (2 N^2), diag(R^H R) (N)
  if (t != 0) return;
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) {
      S.g0r[i * BI_MAXN + j] = sum[2 * (i * N + j)];
      S.g0i[i * BI_MAXN + j] = sum[2 * (i * N + j) + 1];
    }
  if (mode == BS_RES) S.count += 1;
  bool all = true;
  for (int i = 0; i < N; ++i) {
    S.rnorm2[i] = sum[2 * N * N + i];
    S.done[i] = !(S.rnorm2[i] > tol2 * S.bnorm2[i]);
    if (mode == BS_RES && kind == BI_PLAIN && S.done[i]) S.frozen[i] = 1;
    all = all && S.done[i];
  }
  if (mode == BS_INIT) {
    // a (re)start: the plain form freezes exactly the columns that are done
    S.breakdown = 0;
    for (int i = 0; i < N; ++i) S.frozen[i] = kind == BI_PLAIN ? S.done[i] : 0;
    return;
  }
  if (all && S.converged < 0) S.converged = S.count;
}

// |b_i|^2 from the diagonal of a GRAM_FULL partial set (B^H B); clears the state
template <int N>
__global__ void bi_bnorm_kernel(const double* part, int nparts, BiState* st) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  constexpr int nv = 2 * N * N;
  for (int i = wv; i < N; i += 4) {
    const int v = 2 * (i * N + i);
    double s = 0.0;
    for (int b = lane; b < nparts; b += 64) s += part[(long)b * nv + v];
    s = wave_sum(s);
    if (lane == 0) st->bnorm2[i] = s;
  }
  if (threadIdx.x == 0) {
    st->count = 0;
    st->converged = -1;
    for (int i = 0; i < BI_MAXN; ++i) st->frozen[i] = 0;
  }
}

#define BI_N_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
static_assert(BI_MAXN == 8, "one kernel instance per block size 1..BI_MAXN");

template <typename S>
struct BiKernels {
  static hipError_t gram_full(int n, dim3 grid, hipStream_t st, const Geom& g, Field<S> A, Field<S> B, double* part) {
    switch (n) {
#define BI_G(N)                                                                                          \
  case N:                                                                                                \
    hipLaunchKernelGGL((bi_gram_kernel<N, GRAM_FULL, S>), grid, dim3(256), 0, st, g, A, B, A, part);     \
    break;
      BI_N_CASES(BI_G)
#undef BI_G
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  static hipError_t gram_ts(int n, dim3 grid, hipStream_t st, const Geom& g, Field<S> T, Field<S> Sf, Field<S> Rt,
                            double* part) {
    switch (n) {
#define BI_G(N)                                                                                          \
  case N:                                                                                                \
    hipLaunchKernelGGL((bi_gram_kernel<N, GRAM_TS, S>), grid, dim3(256), 0, st, g, T, Sf, Rt, part);     \
    break;
      BI_N_CASES(BI_G)
#undef BI_G
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  static hipError_t s_update(int n, dim3 grid, hipStream_t st, const Geom& g, Field<S> R, Field<S> V, Field<S> Sf,
                             const BiState* state) {
    switch (n) {
#define BI_K(N)                                                                                  \
  case N:                                                                                        \
    hipLaunchKernelGGL((bi_s_kernel<N, S>), grid, dim3(256), 0, st, g, R, V, Sf, state);         \
    break;
      BI_N_CASES(BI_K)
#undef BI_K
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  static hipError_t xr_update(int n, dim3 grid, hipStream_t st, const Geom& g, Field<S> X, Field<S> R, Field<S> Ph,
                              Field<S> Sf, Field<S> Sh, Field<S> T, Field<S> Rt, const BiState* state,
                              double* part) {
    switch (n) {
#define BI_K(N)                                                                                                  \
  case N:                                                                                                        \
    hipLaunchKernelGGL((bi_xr_kernel<N, S>), grid, dim3(256), 0, st, g, X, R, Ph, Sf, Sh, T, Rt, state, part);   \
    break;
      BI_N_CASES(BI_K)
#undef BI_K
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  static hipError_t p_update(int n, dim3 grid, hipStream_t st, const Geom& g, Field<S> R, Field<S> P, Field<S> V,
                             const BiState* state) {
    switch (n) {
#define BI_K(N)                                                                                  \
  case N:                                                                                        \
    hipLaunchKernelGGL((bi_p_kernel<N, S>), grid, dim3(256), 0, st, g, R, P, V, state);          \
    break;
      BI_N_CASES(BI_K)
#undef BI_K
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
};

hipError_t bi_small(int n, hipStream_t st, const double* part, int nparts, int mode, int kind, double tol2,
                    BiState* S) {
  switch (n) {
#define BI_K(N)                                                                                                \
  case N:                                                                                                      \
    hipLaunchKernelGGL((bi_small_kernel<N>), dim3(1), dim3(256), 0, st, part, nparts, mode, kind, tol2, S);    \
    break;
    BI_N_CASES(BI_K)
#undef BI_K
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t bi_bnorm(int n, hipStream_t st, const double* part, int nparts, BiState* S) {
  switch (n) {
#define BI_K(N)                                                                        \
  case N:                                                                              \
    hipLaunchKernelGGL((bi_bnorm_kernel<N>), dim3(1), dim3(256), 0, st, part, nparts, S); \
    break;
    BI_N_CASES(BI_K)
#undef BI_K
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------- driver
// One BiCGStab solver instance in storage S: its fields (even sites; the odd
// halves of V and T are operator scratch), state, partial sums and captured
// iteration graph, kept across calls (the inner solver runs twice per outer
// iteration).
template <typename S>
struct BiSolver {
  OwnedField<S> x, r, rt, p, v, s, t, ph, sh, b;
  DevBuf stb, partb;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  int gk = 0;
  bool precond = false;
  hipError_t alloc(const Geom& g, int n, bool pc) {
    precond = pc;
    for (auto* f : {&x, &r, &rt, &p, &v, &s, &t, &b})
      if (hipError_t e = f->alloc(g, n)) return e;
    if (pc)
      for (auto* f : {&ph, &sh})
        if (hipError_t e = f->alloc(g, n)) return e;
    const int nparts = ((g.vh + 255) / 256) * Store<S>::NC;
    if (hipError_t e = ensure(stb, sizeof(BiState))) return e;
    return ensure(partb, sizeof(double) * (size_t)nparts * (3 * BI_MAXN + 2 * BI_MAXN * BI_MAXN));
  }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    gk = 0;
  }
  ~BiSolver() {
    drop_graph();
    for (auto* f : {&x, &r, &rt, &p, &v, &s, &t, &ph, &sh, &b}) f->free_all();
    release(stb);
    release(partb);
  }
};

template <typename S>
Links<S> links_of(mfq_handle* h);
template <>
Links<double> links_of<double>(mfq_handle* h) {
  return links_d(h);
}
template <>
Links<float> links_of<float>(mfq_handle* h) {
  return links_f(h);
}

struct BiResult {
  int iters = 0, restarts = 0, status = MFQ_OK;
  std::vector<double> rel;  // final relative residual per column (true if measured)
};

// D^ X = B for the n columns of B (even sites), from X = 0.  precond (used
// when the solver has P^, S^ fields) applies K^-1 from one FP64 field into
// another.  Polls the recursive residuals every few iterations; with
// true_check the true residual is then measured and the iteration restarts
// from it (new shadow block) if it lied or broke down, at most max_restarts
// times.
template <typename S, typename PC>
int run_bicgstab(mfq_handle* h, int n, int kind, BiSolver<S>& B, double tol, int max_iter, bool true_check,
                 int max_restarts, PC&& precond, hipStream_t st, BiResult& res) {
  Geom ge = h->g;
  ge.npar = 1;
  const Geom& g = h->g;
  const int nblk = (ge.vh + 255) / 256;
  const dim3 grid(nblk, Store<S>::NC);
  const int nparts = nblk * Store<S>::NC;
  BiState* Sd = (BiState*)B.stb.ptr;
  double* part = (double*)B.partb.ptr;
  Field<S> X = B.x.view(g), R = B.r.view(g), Rt = B.rt.view(g), P = B.p.view(g), V = B.v.view(g),
           Sf = B.s.view(g), T = B.t.view(g), Bf = B.b.view(g);
  const bool use_pc = B.precond;
  Field<S> Ph = use_pc ? B.ph.view(g) : P, Sh = use_pc ? B.sh.view(g) : Sf;
  const Shape sh1 = default_shape(n);
  const double k2 = -h->lat.kappa * h->lat.kappa;
  const double tol2 = tol * tol;
  HopArgs<S, S> a = hop_args<S, S>(h, links_of<S>(h), n);
  // out_e = D^ in_e; out_o = H_oe in_e is the intermediate
  auto apply_a = [&](Field<S> in, Field<S> out, hipStream_t s) -> int {
    a.in = in;
    a.out = out;
    a.par = 1;
    a.coef = 1.0;
    HIPCHK(launch_hop<S, S>(EPI_HOP, a, sh1, s));
    a.in = out;
    a.self = in;
    a.par = 0;
    a.coef = k2;
    HIPCHK(launch_hop<S, S>(EPI_D, a, sh1, s));
    return MFQ_OK;
  };
  auto combine = [&](Field<S> x, Field<S> y, Field<S> out, int sub) -> int {
    hipLaunchKernelGGL((bi_combine_kernel<S>), grid, dim3(256), 0, st, ge, x, y, out, n, sub);
    HIPCHK(hipGetLastError());
    return MFQ_OK;
  };
  BiState host;
  auto poll = [&]() -> int {
    HIPCHK(hipMemcpyAsync(&host, Sd, sizeof(BiState), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    return MFQ_OK;
  };
  // (re)start: R = B - A X (R = B for X = 0), R~ = R, P = R; R~^H R and
  // diag(R^H R) through the update kernel's reduction with alpha = omega = 0
  // (then it leaves X and R as they are)
  auto start = [&](bool zero_x) -> int {
    if (zero_x) {
      HIPCHK(hipMemsetAsync(X.data, 0, field_chunks<S>(g, n) * sizeof(typename Store<S>::chunk), st));
      if (int rc = combine(Bf, Bf, R, 0)) return rc;
    } else {
      if (int rc = apply_a(X, T, st)) return rc;
      if (int rc = combine(Bf, T, R, 1)) return rc;
    }
    if (int rc = combine(R, R, Rt, 0)) return rc;
    if (int rc = combine(R, R, P, 0)) return rc;
    unsigned char* base = (unsigned char*)Sd;
    HIPCHK(hipMemsetAsync(base + offsetof(BiState, ar), 0, 2 * sizeof(double) * BI_MAXN * BI_MAXN, st));
    HIPCHK(hipMemsetAsync(base + offsetof(BiState, wr), 0, 2 * sizeof(double) * BI_MAXN, st));
    HIPCHK(BiKernels<S>::xr_update(n, grid, st, ge, X, R, P, R, R, R, Rt, Sd, part));
    HIPCHK(bi_small(n, st, part, nparts, BS_INIT, kind, tol2, Sd));
    return MFQ_OK;
  };
  res.rel.assign(n, 0.0);
  HIPCHK(hipMemsetAsync(Sd, 0, sizeof(BiState), st));
  HIPCHK(BiKernels<S>::gram_full(n, grid, st, ge, Bf, Bf, part));
  HIPCHK(bi_bnorm(n, st, part, nparts, Sd));
  if (int rc = start(true)) return rc;
  auto iteration = [&](hipStream_t s) -> int {
    if (use_pc)
      if (int r2 = precond(P, Ph)) return r2;
    if (int r2 = apply_a(Ph, V, s)) return r2;
    HIPCHK(BiKernels<S>::gram_full(n, grid, s, ge, Rt, V, part));
    HIPCHK(bi_small(n, s, part, nparts, BS_ALPHA, kind, tol2, Sd));
    HIPCHK(BiKernels<S>::s_update(n, grid, s, ge, R, V, Sf, Sd));
    if (use_pc)
      if (int r2 = precond(Sf, Sh)) return r2;
    if (int r2 = apply_a(Sh, T, s)) return r2;
    HIPCHK(BiKernels<S>::gram_ts(n, grid, s, ge, T, Sf, Rt, part));
    HIPCHK(bi_small(n, s, part, nparts, BS_OMEGA, kind, tol2, Sd));
    HIPCHK(BiKernels<S>::xr_update(n, grid, s, ge, X, R, Ph, Sf, Sh, T, Rt, Sd, part));
    HIPCHK(bi_small(n, s, part, nparts, BS_RES, kind, tol2, Sd));
    HIPCHK(BiKernels<S>::p_update(n, grid, s, ge, R, P, V, Sd));
    return MFQ_OK;
  };
  // without a preconditioner, k iterations are captured once and replayed
  // between polls; with one, every iteration polls (its inner solves do)
  const int every = use_pc ? 1 : 4;
  int iters = 0, rc = MFQ_OK;
  for (;;) {
    while (iters < max_iter) {
      const int k = every < max_iter - iters ? every : max_iter - iters;
      if (!use_pc && k == every) {
        if (!B.gexec || B.gk != k) {
          B.drop_graph();
          HIPCHK(hipStreamBeginCapture(h->cap_stream, hipStreamCaptureModeThreadLocal));
          int rc2 = MFQ_OK;
          for (int i = 0; i < k && rc2 == MFQ_OK; ++i) rc2 = iteration(h->cap_stream);
          hipError_t ec = hipStreamEndCapture(h->cap_stream, &B.graph);
          if (rc2 != MFQ_OK) return rc2;
          HIPCHK(ec);
          HIPCHK(hipGraphInstantiate(&B.gexec, B.graph, nullptr, nullptr, 0));
          B.gk = k;
        }
        HIPCHK(hipGraphLaunch(B.gexec, st));
      } else {
        for (int i = 0; i < k; ++i)
          if ((rc = iteration(st))) return rc;
      }
      iters += k;
      if ((rc = poll())) return rc;
      bool all = true;
      for (int i = 0; i < n; ++i) all = all && host.done[i];
      if (all || host.breakdown) break;
    }
    if (!true_check) {
      bool all = true;
      for (int i = 0; i < n; ++i) {
        res.rel[i] = host.bnorm2[i] > 0 ? sqrt(host.rnorm2[i] / host.bnorm2[i]) : 0.0;
        all = all && host.done[i];
      }
      res.status = all ? MFQ_OK : MFQ_NOT_CONVERGED;
      break;
    }
    // measure the true residual; restart from it unless every column is done
    const int conv = host.converged;
    if ((rc = start(false))) return rc;
    if ((rc = poll())) return rc;
    bool all = true;
    for (int i = 0; i < n; ++i) {
      res.rel[i] = host.bnorm2[i] > 0 ? sqrt(host.rnorm2[i] / host.bnorm2[i]) : 0.0;
      all = all && host.done[i];
    }
    if (all) {
      host.converged = conv;
      res.status = MFQ_OK;
      break;
    }
    if (iters >= max_iter || res.restarts >= max_restarts) {
      res.status = MFQ_NOT_CONVERGED;
      break;
    }
    res.restarts += 1;
    const int minus1 = -1;
    HIPCHK(hipMemcpyAsync((unsigned char*)Sd + offsetof(BiState, converged), &minus1, sizeof(int),
                          hipMemcpyHostToDevice, st));
  }
  // iterations until every column first met the tolerance (polls come every
  // few iterations, so the loop may have run a few more)
  res.iters = host.converged >= 0 && host.converged <= host.count ? host.converged : host.count;
  return MFQ_OK;
}

// The paper's form: D^ x_e = b_e for the n columns in ws.b64 (even sites),
// solution into ws.x64 (even sites), kind = plain / global / block BiCGStab in
// FP64, with an FP32 inner BiCGStab per column as the right preconditioner
// when prec is MFQ_PREC_FP32_RELIABLE.
int run_bicgstab_schur(mfq_handle* h, int n, int kind, const mfq_solve_params* P, hipStream_t st,
                       mfq_solve_stats* stats) {
  if (n > BI_MAXN) return fail(MFQ_ERR_ARG, "the BiCGStab solvers take at most 8 right-hand sides");
  if (P->prec != MFQ_PREC_FP64 && P->prec != MFQ_PREC_FP32_RELIABLE)
    return fail(MFQ_ERR_ARG, "the BiCGStab solvers run in FP64, or FP64 outer with an FP32 inner solve");
  const bool pc = P->prec == MFQ_PREC_FP32_RELIABLE;
  if (int rc = need_su3(h, P->prec, MFQ_PC_NONE)) return rc;
  Workspace& w = h->ws;
  const Geom& g = h->g;
  Geom ge = g;
  ge.npar = 1;
  BiSolver<double> outer;
  BiSolver<float> inner;
  if (outer.alloc(g, n, pc) != hipSuccess || (pc && inner.alloc(g, n, false) != hipSuccess))
    return fail(MFQ_ERR_NOMEM, "BiCGStab fields");
  const Shape sh1 = default_shape(n);
  HIPCHK(launch_convert<double, double>(ge, w.b64.view(g), outer.b.view(g), 0, n, sh1, st));
  const double inner_tol = P->inner_tol > 0.0 ? P->inner_tol : 1e-4;
  const int inner_max = P->inner_max_iter > 0 ? P->inner_max_iter : 500;
  long inner_iters = 0;
  int inner_calls = 0;
  // K^-1 in = the FP32 BiCGStab solution of D^ z = in, per column, from z = 0
  auto precond = [&](Field<double> in, Field<double> out) -> int {
    HIPCHK(launch_convert<double, float>(ge, in, inner.b.view(g), 0, n, sh1, st));
    BiResult ir;
    auto none = [](Field<float>, Field<float>) -> int { return MFQ_OK; };
    if (int r2 = run_bicgstab<float>(h, n, BI_PLAIN, inner, inner_tol, inner_max, false, 0, none, st, ir)) return r2;
    inner_iters += ir.iters;
    inner_calls += 1;
    HIPCHK(launch_convert<float, double>(ge, inner.x.view(g), out, 0, n, sh1, st));
    return MFQ_OK;
  };
  BiResult res;
  if (int rc = run_bicgstab<double>(h, n, kind, outer, P->tol, P->max_iter, true, 5, precond, st, res)) return rc;
  HIPCHK(launch_convert<double, double>(ge, outer.x.view(g), w.x64.view(g), 0, n, sh1, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int i = 0; stats && i < n; ++i) {
    stats[i].iters = res.iters;
    stats[i].reliable_updates = res.restarts;
    stats[i].true_rel_resid = res.rel[i];
    stats[i].status = res.rel[i] <= P->tol ? MFQ_OK : MFQ_NOT_CONVERGED;
    stats[i].inner_iters = (int)inner_iters;
    stats[i].inner_calls = inner_calls;
  }
  return res.status;
}

}  // namespace mfq
