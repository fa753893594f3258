// The library handle and the host-side helpers shared by the translation
// units that drive solves (single lattice and multi-lattice batch).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "internal.h"
#include "mfq.h"

namespace mfq {

struct Workspace {
  OwnedField<double> b64, x64, r64, t64, y64;
  OwnedField<double> aux64;  // route S force: X while Y is solved for
  OwnedField<double> xd, rd, pd, td;
  OwnedField<float> xs, rs, ps, ts;
  OwnedField<_Float16> rh, ph, th;
  DevBuf part, sc, sums, bad;
  DevBuf md_part, md_u0, md_p0, md_force;  // molecular dynamics (md.hip)
  // FGMRES (fgmres.hip): basis, preconditioned directions, A z, the CG
  // fallback's saved x and b, per-RHS state, partial sums; kept between calls
  // so that a captured cycle can be replayed by the next solve
  DevBuf gm_v, gm_z, gm_w, gm_xsave, gm_bsave, gm_st, gm_part;
  int cap_part = 0;  // RHS capacity of the partial-sum slots
  int nblk_max = 0;
  CgScalars* host_sc = nullptr;
  int host_cap = 0;
};

// A captured run of k inner CG iterations.  The key holds everything the
// captured kernel arguments depend on, so a stale graph never matches.
struct GraphEntry {
  std::vector<uintptr_t> key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// Learned-preconditioner state (allocated on first use).
struct PtcState {
  DevBuf w_master;  // FP32 master weights: W1 then W2, interleaved complex
  DevBuf w_infer;   // the same rounded to BF16 values (inference weights)
  DevBuf adam_m, adam_v, grad, part, enorm2;
  OwnedField<float> hid, y, gy, gh;
  OwnedField<double> pr, pe;  // packed training pairs (residuals, errors)
  DevBuf ops, chi;  // matrix-core weight operands; layer-2 mixings before transport
  DevBuf ops_train, ops_adj, wadj;  // training: hi/lo operands of the master and the adjoint weights
  int adam_t = 0;
  int w_version = 0, ops_version = -1;  // ops are rebuilt when the inference weights change
  bool have_weights = false;
};

struct TuneEntry {
  int n, prec;
  Shape sh;
  float us;
};

}  // namespace mfq

struct mfq_handle {
  std::vector<mfq::TuneEntry> tuned;  // autotuned launch shapes, by (n_rhs, precision)
  int autotune = 1;
  mfq_lattice lat;
  mfq::Geom g;
  int n_slices;
  mfq::DevBuf links64, links32, links16;
  mfq::Workspace ws;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  hipStream_t cap_stream = nullptr;  // used only to capture graphs
  std::vector<mfq::GraphEntry> graphs;
  mfq::PtcState* ptc = nullptr;
  int links_su3 = 0;  // every link is SU(3): the two-row FP32 / FP16 copies are valid
};


namespace mfq {

int fail(int code, const std::string& msg);
int fail_hip(hipError_t e, const char* what);
uintptr_t bits(double v);
void drop_graphs(mfq_handle* h);
Links<double> links_d(mfq_handle* h);
Links<float> links_f(mfq_handle* h);
Links<_Float16> links_h(mfq_handle* h);
int partials_ready(mfq_handle* h, int n_rhs);
double* part_slot(mfq_handle* h, int slot);
int ensure_fp64_fields(mfq_handle* h, int n);
int check_params(const mfq_solve_params* P);
int need_su3(mfq_handle* h, int prec, int precond);
int pack_checked(mfq_handle* h, const double* canon, int n_rhs, int gamma5, hipStream_t st);
int solve_packed(mfq_handle* h, int n, const mfq_solve_params* P, hipStream_t st, mfq_solve_stats* stats,
                 bool schur = false);
// D z = b (dagger 0) or D^+ z = b (dagger 1) through the even/odd Schur
// complement: b in ws.b64, z in ws.x64 (b64, r64, t64, y64 overwritten)
int schur_solve(mfq_handle* h, int n, int dagger, const mfq_solve_params* P, hipStream_t st,
                mfq_solve_stats* stats);
void merge_stats(mfq_solve_stats* a, const mfq_solve_stats* b, int n);
// the paper's BiCGStab solvers on the even/odd system (bicgstab.hip): D^ x_e =
// b_e for b in ws.b64, x into ws.x64 (even sites); kind 0 plain, 1 global, 2 block
int run_bicgstab_schur(mfq_handle* h, int n, int kind, const mfq_solve_params* P, hipStream_t st,
                       mfq_solve_stats* stats);
inline bool is_bicgstab(int precond) {
  return precond == MFQ_PC_BICGSTAB || precond == MFQ_PC_GL_BICGSTAB || precond == MFQ_PC_BL_BICGSTAB;
}
inline int bicgstab_kind(int precond) { return precond - MFQ_PC_BICGSTAB; }
// per-RHS FP64 |b - D^+D x| / |b| into stats[].true_rel_resid (b in b64, x in x64)
int full_residual(mfq_handle* h, int n, hipStream_t st, mfq_solve_stats* stats);
// flexible GMRES with the learned (or identity) preconditioner (fgmres.hip)
int run_fgmres(mfq_handle* h, int n, const mfq_solve_params* P, hipStream_t st, mfq_solve_stats* stats);
int run_block_cg(mfq_handle* h, int n, const mfq_solve_params* P, hipStream_t st, mfq_solve_stats* stats);
// the tuned launch shape of the FP64 hopping kernel for n RHS
int fp64_hop_shape(mfq_handle* h, int n, hipStream_t st, Shape* out);
// The tuned FP32 shape (allocates the FP32 p and t fields of the workspace,
// which it times on; t then serves as scratch of the FP32 operator).
int fp32_hop_shape(mfq_handle* h, int n, hipStream_t st, Shape* out);
// out = op(in) in FP64 (mfq_op); tmp is scratch for DDAGD; sh2 is the shape of
// the both-parity launches
int apply_op_fp64(mfq_handle* h, int op, Field<double> in, Field<double> tmp, Field<double> out, int n_rhs,
                  Shape sh2, hipStream_t st);
// the per-device address of the no-allocation entry point's workspace
int noalloc_init_current_device();
// learned preconditioner (ptc_host.hip)
void ptc_free(mfq_handle* h);
template <typename S>
int ptc_apply_fields(mfq_handle* h, Field<S> in, Field<S> out, int n, hipStream_t st);
// the same in two parts: the weight operands and the n-RHS scratch made
// ready (may allocate), then the launches alone (nothing allocated: safe
// inside a graph capture once ptc_prepare has run for n)
int ptc_prepare(mfq_handle* h, int n, hipStream_t st);
template <typename S>
int ptc_launch_fields(mfq_handle* h, Field<S> in, Field<S> out, int n, hipStream_t st);

template <typename S, typename SX>
HopArgs<S, SX> hop_args(mfq_handle* h, Links<S> L, int n_rhs) {
  HopArgs<S, SX> a;
  memset((void*)&a, 0, sizeof(a));
  a.g = h->g;
  a.links = L;
  a.n_rhs = n_rhs;
  a.skip_state = 3;
  a.upd_mode = -1;
  return a;
}

}  // namespace mfq

#define HIPCHK(...)                                          \
  do {                                                       \
    hipError_t e_ = (__VA_ARGS__);                           \
    if (e_ != hipSuccess) return fail_hip(e_, #__VA_ARGS__); \
  } while (0)
