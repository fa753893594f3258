// Host-side internals shared by the translation units of libmfq: kernel
// launchers, the solver state that lives in device memory, and the handle.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "device.h"

namespace mfq {

// ----------------------------------------------------------- CG scalars
// One record per right-hand side, in device memory.  Double-buffered copies
// are not needed because every scalar update happens in a one-block
// finishing kernel between the vector kernels.
// ST_WAIT: the residual dropped by delta since the last true residual; the
// RHS pauses until the reliable update (so that the update is never late),
// keeping its search direction.  ST_CHECK: the recursion claims convergence
// (or broke down); the update checks the truth and restarts p.
enum : int { ST_ACTIVE = 0, ST_WAIT = 1, ST_CHECK = 2, ST_DONE = 3 };

struct CgScalars {
  double rho;     // |r|^2 of the current (inner) residual
  double rho_ru;  // |r|^2 at the last reliable update
  double bnorm2;  // |b|^2
  double alpha, beta, pap;
  double rtrue2;  // |b - A x|^2 at the last true-residual evaluation
  double pad;
  int state;  // ST_ACTIVE, ST_CHECK (needs a true-residual check), ST_DONE
  int iters;
  int pad1;
  int n_true; // true-residual evaluations
  int rp;     // at the next restart: 1 p = r, 2 p = r + beta p, 0 keep p
  int fresh;  // the last true-residual evaluation covered this RHS: reload r
};

// Which RHS a reliable update covers: every unfinished one (UPD_ALL), or only
// those that asked for it (UPD_FLAGGED: ST_WAIT or ST_CHECK), so that RHS and
// lattices sharing one solve keep their own update schedule.
enum : int { UPD_ALL = 0, UPD_FLAGGED = 1 };

__host__ __device__ inline bool in_update(const CgScalars& s, int mode) {
  return s.state != ST_DONE && (mode == UPD_ALL || s.state == ST_WAIT || s.state == ST_CHECK);
}

enum : int {
  FIN_STORE = 0,  // out[r] = sum
  FIN_ALPHA = 1,  // pap = sum; alpha = rho / pap
  FIN_BETA = 2,   // rho' = sum; beta = rho'/rho; convergence / update flags
  FIN_TRUE = 3,   // true residual (every unfinished RHS): done, or restart the recursion from it
  FIN_INIT = 4,   // |b|^2: initial state
  FIN_TRUE_FLAGGED = 5,  // as FIN_TRUE, for the RHS that asked for an update only
};

// Epilogues of the hopping kernel.
enum : int {
  EPI_HOP = 0,    // out = b * (H in)
  EPI_D = 1,      // out = self + b * (H in) [+ partial |out|^2]
  EPI_CGUPD = 2,  // ap = self + b * (H in); r -= alpha ap; x += alpha p; partial |r|^2
  EPI_RES = 3,    // r64 = bvec - (self + b * (H in)); partial |r64|^2  (FP64)
};

struct Partials {
  double* part;  // [n_rhs][nblk]
  int nblk;
};

// Launch shape of the site x RHS kernels.
struct Shape {
  int sb;   // sites per workgroup (multiple of 64)
  int nr;   // right-hand sides per workgroup
  int xcd;  // bit 0: remap workgroups so each XCD walks a contiguous chunk of
            // tiles; bit 1: z-blocked tile order (see HopArgs::zb)
  int tc;   // both-parity launches: 0, or each thread sweeps tc time slices of
            // one spatial site (sb spatial sites per workgroup)
  int ds;   // 0, or 2 / 4: the 4 directions of a site split over that many
            // wavefronts of one workgroup (64 sites x nr RHS, ds * nr <= 8)
};

// Upper bound on the workgroups along x of any hopping launch (partial-sum
// capacity per RHS).
int max_hop_blocks(const Geom& g);

Shape default_shape(int n_rhs);
// Workgroups along x of a hopping launch (par 0 / 1, or 2 for both parities).
int hop_grid_x(const Geom& g, Shape sh, int par);

// The hopping kernel, all precisions and epilogues.
template <typename S, typename SX>
struct HopArgs {
  Geom g;
  Links<S> links;
  Field<S> in;         // read at the neighbours (parity 1 - par)
  Field<S> self;       // read at the output site (parity par)
  Field<S> out;        // EPI_HOP / EPI_D output; EPI_CGUPD residual (rmw)
  Field<SX> x;         // EPI_CGUPD solution correction (rmw)
  Field<S> p;          // EPI_CGUPD search direction
  Field<double> bvec;  // EPI_RES right-hand side
  Field<double> r64;   // EPI_RES output
  CgScalars* sc;       // per-RHS scalars (alpha, state) or null
  double* part;        // partial sums [n_rhs][gridDim.x] or null
  const double* apart; // EPI_CGUPD: reduce alpha from these |D p|^2 partials [n_rhs][anblk]
  int anblk;
  int par;             // output parity 0 / 1, or 2 for both parities in one launch
  int n_rhs, dagger, skip_state;
  int upd_mode;        // >= 0: run only the RHS in_update(sc[r], upd_mode); else use skip_state
  int xcd;             // set by the launcher from the Shape
  // z-blocked tile order (0: tiles in half-index order).  Tiles are whole
  // pieces of one (z, t) plane; they are walked plane by plane over zb
  // consecutive z, then t, then the next block of zb z values, so a spinor's
  // and a link's t and z neighbours are read a few dozen tiles apart, inside
  // one XCD's L2, instead of a whole time slice apart.  tpp = tiles per plane.
  int zb, tpp;
  int zbl;             // log2(zb) (zb is 1, 2 or 4)
  unsigned mtpp, mtd;  // division magic (fdiv) of tpp and of the dynamical time extent
  double coef;         // coefficient of the hopping term
};

template <typename S, typename SX>
hipError_t launch_hop(int epi, const HopArgs<S, SX>& a, Shape sh, hipStream_t st);

hipError_t launch_finish(int fin, const Partials* parts, int n_parts, int n_rhs, CgScalars* sc,
                         double* out, double tol2, double delta2, hipStream_t st);

// Vector kernels (both parities, sites x RHS).
template <typename S>
hipError_t launch_xpay_p(const Geom& g, Field<S> r, Field<S> p, const CgScalars* sc, int n_rhs,
                         Shape sh, hipStream_t st);
template <typename SX>
hipError_t launch_fold(const Geom& g, Field<SX> xi, Field<double> x64, const CgScalars* sc,
                       int n_rhs, int mode, Shape sh, hipStream_t st);
template <typename S>
hipError_t launch_restart(const Geom& g, Field<double> r64, Field<S> ri, Field<S> pi,
                          const CgScalars* sc, int n_rhs, Shape sh, hipStream_t st);
template <typename SA, typename SB>
hipError_t launch_convert(const Geom& g, Field<SA> src, Field<SB> dst, int gamma5, int n_rhs,
                          Shape sh, hipStream_t st);
hipError_t launch_norm2(const Geom& g, Field<double> f, double* part, int n_rhs, Shape sh,
                        int nblk, hipStream_t st);
// zero parity `par` of every RHS of f (values and, for FP16, norms)
template <typename S>
hipError_t launch_zero_parity(const Geom& g, Field<S> f, int n_rhs, int par, hipStream_t st);
hipError_t launch_fill_pattern(const Geom& g, Field<double> f, int n_rhs, Shape sh, hipStream_t st);
hipError_t launch_init_residual(const Geom& g, Field<double> b, Field<double> r64, double* part,
                                int n_rhs, Shape sh, hipStream_t st);

// Canonical <-> internal layout.
template <typename S>
hipError_t launch_pack_spinor(const Geom& g, const double* canon, Field<S> f, int n_rhs, int gamma5,
                              int* bad_flag, hipStream_t st);
hipError_t launch_unpack_spinor(const Geom& g, Field<double> f, double* canon, int n_rhs,
                                hipStream_t st);
template <typename S>
hipError_t launch_pack_links(const Geom& g, const double* canon, typename Store<S>::link_elem* out,
                             int* bad_flag, int comp, int su3_check, hipStream_t st);

// Fermion force: G_mu(n) summed over RHS, canonical FP64 output.
hipError_t launch_force(const Geom& g, Links<double> links, Field<double> X, Field<double> Y,
                        int n_rhs, double kappa, double* force_canon, int n_link_slices,
                        hipStream_t st);

// ------------------------------------------------------------- buffers
struct DevBuf {
  void* ptr = nullptr;
  size_t bytes = 0;
};

hipError_t ensure(DevBuf& b, size_t bytes);
void release(DevBuf& b);

template <typename S>
size_t field_chunks(const Geom& g, int n_rhs) {
  return (size_t)n_rhs * 2 * Store<S>::NC * g.vs;
}

template <typename S>
struct OwnedField {
  DevBuf data, norm;
  hipError_t alloc(const Geom& g, int n_rhs) {
    hipError_t e = ensure(data, field_chunks<S>(g, n_rhs) * sizeof(typename Store<S>::chunk));
    if (e != hipSuccess) return e;
    if (sizeof(S) == 2) return ensure(norm, (size_t)n_rhs * 2 * g.vs * sizeof(float));
    return hipSuccess;
  }
  Field<S> view(const Geom& g) const {
    Field<S> f;
    f.data = (typename Store<S>::chunk*)data.ptr;
    f.norm = (float*)norm.ptr;
    f.vh = g.vs;
    return f;
  }
  void free_all() {
    release(data);
    release(norm);
  }
};

}  // namespace mfq
