// Molecular dynamics of the many-flavor HMC on the GPU (Section 2: the
// pseudo-fermion action of Eq. 2 in a hybrid Monte Carlo with the force of
// Eq. 3): momentum and link updates of the leapfrog integrator, the kinetic
// energy in FP64, and one whole trajectory with its FP64 Delta H and the
// Metropolis decision.
//
// Momenta are stored like the force: the Hermitian traceless matrix
// P_mu(n) = sum_a P^a_mu(n) T^a per link, canonical link layout, FP64.  The
// equations of motion are dU/dt = i P U and dP/dt = -G (G the force of
// mfq_fermion_force); H = 1/2 sum P^a P^a + sum_i |D^-1 phi_i|^2, where
// 1/2 sum_a P^a P^a = Tr P^2 = sum_ij |P_ij|^2.  Only the links that enter
// D move (under Schroedinger-functional boundaries the spatial links at
// x0 = 0, T and the temporal links at x0 = 0, T-1 and T do not): the others
// keep their link and are left out of the kinetic energy.
#include <math.h>
#include <string.h>

#include <chrono>

#include "handle.h"

namespace mfq {

struct LinkGeom {
  int lx, ly, lz, ns;  // spatial extents, stored time slices
  int sf, t;           // Schroedinger-functional boundaries, T
  long nlinks;         // 4 * ns * lx * ly * lz
};

static LinkGeom link_geom(const mfq_handle* h) {
  LinkGeom lg;
  lg.lx = h->lat.dims[0];
  lg.ly = h->lat.dims[1];
  lg.lz = h->lat.dims[2];
  lg.t = h->lat.dims[3];
  lg.ns = h->n_slices;
  lg.sf = h->lat.bc == MFQ_BC_SF;
  lg.nlinks = 4L * lg.ns * lg.lx * lg.ly * lg.lz;
  return lg;
}

// Does link l (canonical index [mu][x0][z][y][x]) enter D?
__device__ __forceinline__ bool link_enters(const LinkGeom& lg, long l) {
  if (!lg.sf) return true;
  const long per_slice = (long)lg.lx * lg.ly * lg.lz;
  const int x0 = (int)((l / per_slice) % lg.ns);
  const int mu = (int)(l / (per_slice * lg.ns));
  return mu == 0 ? (x0 >= 1 && x0 <= lg.t - 2) : (x0 >= 1 && x0 <= lg.t - 1);
}

typedef cpx<double> c64;

__device__ __forceinline__ void load3(const d2* p, c64 m[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = {p[k].x, p[k].y};
}
__device__ __forceinline__ void store3(d2* p, const c64 m[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    d2 q;
    q.x = m[k].re;
    q.y = m[k].im;
    p[k] = q;
  }
}
// c = a b
__device__ __forceinline__ void mul3(const c64 a[9], const c64 b[9], c64 c[9]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = cmul(a[3 * i], b[j]) + cmul(a[3 * i + 1], b[3 + j]) + cmul(a[3 * i + 2], b[6 + j]);
}

// exp(A) of a 3x3 complex matrix with |A| modest (here A = i eps P): scaling
// by 2^-s until the max-row-sum norm is <= 1/8, a degree-12 Taylor
// polynomial in Horner form (truncation < 1e-21 relative), and s squarings.
__device__ void expm3(const c64 a_in[9], c64 e[9]) {
  c64 a[9];
  double nrm = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double r = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j) r += sqrt(norm2(a_in[3 * i + j]));
    nrm = fmax(nrm, r);
  }
  int s = 0;
  while (nrm > 0.125 && s < 60) {
    nrm *= 0.5;
    ++s;
  }
  const double sc = ldexp(1.0, -s);
#pragma unroll
  for (int k = 0; k < 9; ++k) a[k] = sc * a_in[k];
  // M = I + A/12; M = I + (A/j) M for j = 11..1
  c64 m[9], t[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = (1.0 / 12.0) * a[k];
  m[0].re += 1.0;
  m[4].re += 1.0;
  m[8].re += 1.0;
  for (int j = 11; j >= 1; --j) {
    mul3(a, m, t);
    const double inv = 1.0 / j;
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = inv * t[k];
    m[0].re += 1.0;
    m[4].re += 1.0;
    m[8].re += 1.0;
  }
  for (int q = 0; q < s; ++q) {
    mul3(m, m, t);
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = t[k];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) e[k] = m[k];
}

// P <- P - eps G on the links that enter D.
__global__ void md_momenta_kernel(LinkGeom lg, const d2* g, d2* p, double eps) {
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= lg.nlinks || !link_enters(lg, l)) return;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    d2 v = p[9 * l + k];
    const d2 f = g[9 * l + k];
    v.x -= eps * f.x;
    v.y -= eps * f.y;
    p[9 * l + k] = v;
  }
}

// U <- exp(i eps P) U on the links that enter D.
__global__ void md_links_kernel(LinkGeom lg, const d2* p, d2* u, double eps) {
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= lg.nlinks || !link_enters(lg, l)) return;
  c64 a[9], e[9], uu[9], out[9];
  load3(p + 9 * l, a);
#pragma unroll
  for (int k = 0; k < 9; ++k) a[k] = eps * imul(a[k]);
  expm3(a, e);
  load3(u + 9 * l, uu);
  mul3(e, uu, out);
  store3(u + 9 * l, out);
}

// Partial sums of Tr P^2 = sum_ij |P_ij|^2 over the links that enter D, one
// per workgroup (256 threads).
__global__ __launch_bounds__(256) void md_kinetic_kernel(LinkGeom lg, const d2* p, double* part) {
  const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
  double v = 0.0;
  if (l < lg.nlinks && link_enters(lg, l)) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const d2 q = p[9 * l + k];
      v += q.x * q.x + q.y * q.y;
    }
  }
  __shared__ double ws[4];
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = ((ws[0] + ws[1]) + ws[2]) + ws[3];
}

static int md_blocks(const LinkGeom& lg) { return (int)((lg.nlinks + 255) / 256); }

int kinetic_energy(mfq_handle* h, const double* mom_dev, double* out, hipStream_t st) {
  const LinkGeom lg = link_geom(h);
  const int nb = md_blocks(lg);
  Workspace& w = h->ws;
  HIPCHK(ensure(w.md_part, sizeof(double) * (nb + 1)));
  double* part = (double*)w.md_part.ptr;
  hipLaunchKernelGGL(md_kinetic_kernel, dim3(nb), dim3(256), 0, st, lg, (const d2*)mom_dev, part);
  HIPCHK(hipGetLastError());
  Partials pp{part, nb};
  HIPCHK(launch_finish(FIN_STORE, &pp, 1, 1, nullptr, part + nb, 0.0, 0.0, st));
  HIPCHK(hipMemcpyAsync(out, part + nb, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  return MFQ_OK;
}

int md_momenta(mfq_handle* h, const double* force_dev, double* mom_dev, double eps, hipStream_t st) {
  const LinkGeom lg = link_geom(h);
  hipLaunchKernelGGL(md_momenta_kernel, dim3(md_blocks(lg)), dim3(256), 0, st, lg, (const d2*)force_dev,
                     (d2*)mom_dev, eps);
  HIPCHK(hipGetLastError());
  return MFQ_OK;
}

int md_links(mfq_handle* h, const double* mom_dev, double* links_dev, double eps, hipStream_t st) {
  const LinkGeom lg = link_geom(h);
  hipLaunchKernelGGL(md_links_kernel, dim3(md_blocks(lg)), dim3(256), 0, st, lg, (const d2*)mom_dev,
                     (d2*)links_dev, eps);
  HIPCHK(hipGetLastError());
  return mfq_update_links(h, links_dev, st);  // repack the handle's copies
}

}  // namespace mfq

using namespace mfq;

extern "C" {

int mfq_kinetic_energy(mfq_handle* h, const double* mom_dev, double* out_host, void* stream) {
  if (!h || !mom_dev || !out_host) return fail(MFQ_ERR_ARG, "NULL argument");
  return kinetic_energy(h, mom_dev, out_host, (hipStream_t)stream);
}

int mfq_md_momenta(mfq_handle* h, const double* force_dev, double* mom_dev, double eps, void* stream) {
  if (!h || !force_dev || !mom_dev) return fail(MFQ_ERR_ARG, "NULL argument");
  if (!isfinite(eps)) return fail(MFQ_ERR_ARG, "eps must be finite");
  return md_momenta(h, force_dev, mom_dev, eps, (hipStream_t)stream);
}

int mfq_md_links(mfq_handle* h, const double* mom_dev, double* links_dev, double eps, void* stream) {
  if (!h || !mom_dev || !links_dev) return fail(MFQ_ERR_ARG, "NULL argument");
  if (!isfinite(eps)) return fail(MFQ_ERR_ARG, "eps must be finite");
  return md_links(h, mom_dev, links_dev, eps, (hipStream_t)stream);
}

int mfq_hmc_trajectory(mfq_handle* h, double* links_dev, double* mom_dev, const double* phi_dev, int n_rhs,
                       const mfq_hmc_params* hp, const mfq_solve_params* sp, mfq_hmc_result* out, void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  if (!h || !links_dev || !mom_dev || !phi_dev || !hp || !sp || !out) return fail(MFQ_ERR_ARG, "NULL argument");
  if (n_rhs < 1) return fail(MFQ_ERR_ARG, "n_rhs must be >= 1");
  if (!(hp->tau > 0.0) || !isfinite(hp->tau) || hp->n_steps < 1)
    return fail(MFQ_ERR_ARG, "tau must be > 0 and n_steps >= 1");
  if (!(hp->rand_uniform >= 0.0 && hp->rand_uniform < 1.0))
    return fail(MFQ_ERR_ARG, "rand_uniform must be in [0, 1)");
  hipStream_t st = (hipStream_t)stream;
  memset(out, 0, sizeof(*out));
  Workspace& w = h->ws;
  const LinkGeom lg = link_geom(h);
  const size_t lbytes = (size_t)lg.nlinks * 9 * sizeof(d2);
  HIPCHK(ensure(w.md_u0, lbytes));
  HIPCHK(ensure(w.md_p0, lbytes));
  HIPCHK(ensure(w.md_force, lbytes));
  HIPCHK(hipMemcpyAsync(w.md_u0.ptr, links_dev, lbytes, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(w.md_p0.ptr, mom_dev, lbytes, hipMemcpyDeviceToDevice, st));
  // the handle's packed links must be those of links_dev at the start
  int rc = mfq_update_links(h, links_dev, st);
  if (rc) return rc;
  std::vector<double> act(n_rhs);
  std::vector<mfq_solve_stats> stats(n_rhs);
  double* force = (double*)w.md_force.ptr;
  int worst = MFQ_OK;
  auto eval_force = [&](double* s_sum) -> int {
    const int r = mfq_fermion_force(h, phi_dev, n_rhs, sp, force, act.data(), nullptr, nullptr, stats.data(), st);
    if (r < 0) return r;
    if (r != MFQ_OK) worst = r;
    double s = 0.0;
    for (int i = 0; i < n_rhs; ++i) {
      s += act[i];
      out->solver_iters += stats[i].iters;
    }
    *s_sum = s;
    out->force_evals += 1;
    return MFQ_OK;
  };
  const double dt = hp->tau / hp->n_steps;
  if ((rc = kinetic_energy(h, mom_dev, &out->kinetic_old, st))) return rc;
  double s_now = 0.0;
  if ((rc = eval_force(&out->action_old))) return rc;
  if ((rc = md_momenta(h, force, mom_dev, 0.5 * dt, st))) return rc;
  for (int step = 0; step < hp->n_steps; ++step) {
    if ((rc = md_links(h, mom_dev, links_dev, dt, st))) return rc;
    if ((rc = eval_force(&s_now))) return rc;
    if ((rc = md_momenta(h, force, mom_dev, step + 1 < hp->n_steps ? dt : 0.5 * dt, st))) return rc;
  }
  out->action_new = s_now;
  if ((rc = kinetic_energy(h, mom_dev, &out->kinetic_new, st))) return rc;
  out->delta_h = (out->kinetic_new - out->kinetic_old) + (out->action_new - out->action_old);
  // Metropolis with the caller's uniform draw: accept if u < exp(-dH), compared
  // as log u < -dH so that a large dH (exp underflowing to 0) still accepts
  // the draw u = 0 (log 0 = -inf)
  const double u = hp->rand_uniform;
  out->accepted = isfinite(out->delta_h) && (u == 0.0 || log(u) < -out->delta_h) ? 1 : 0;
  if (!out->accepted) {
    HIPCHK(hipMemcpyAsync(links_dev, w.md_u0.ptr, lbytes, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(mom_dev, w.md_p0.ptr, lbytes, hipMemcpyDeviceToDevice, st));
    if ((rc = mfq_update_links(h, links_dev, st))) return rc;
  }
  HIPCHK(hipStreamSynchronize(st));
  out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return worst;
}

}  // extern "C"
