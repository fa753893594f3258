/* mfq.h -- C ABI of the MI355X many-flavor quark-solve library (libmfq.so).
 *
 * The library computes, for N_f/2 independent pseudo-fermion fields
 * Phi = (phi_1 .. phi_{N_f/2}) on one SU(3) gauge field U with Wilson quarks
 * of hopping parameter kappa, the blocked quantities of the paper's Alg. 2:
 *
 *   X = D^-1 Phi,   Y = (D^+)^-1 X,   F_mu(n) = sum_i f[x_i, y_i]   (Eq. 3)
 *
 * and the pseudo-fermion action S_i = |D^-1 phi_i|^2 (Eq. 2).  The solves are
 * conjugate gradients on the normal operator D^+ D run for all right-hand
 * sides (RHS) at once, so that one link load serves every pseudo-fermion.
 *
 * Conventions (the paper writes none of them out; they are this library's):
 *   (D psi)(n) = psi(n) - kappa sum_mu [ (1 - g_mu) U_mu(n) psi(n+mu)
 *                                        + (1 + g_mu) U_mu(n-mu)^+ psi(n-mu) ],
 *   chiral gamma basis g_mu = [[0, e_mu], [e_mu^+, 0]], e_0 = -1, e_k = -i sigma_k,
 *   g_5 = diag(1, 1, -1, -1), mu = 0 is time, 1..3 are x, y, z.
 *   Schroedinger-functional (SF) time boundaries: slices x0 = 0..T, spinors
 *   vanish on x0 = 0 and x0 = T, so the dynamical slices are x0 = 1..T-1.
 *
 * Canonical boundary layouts (FP64, complex interleaved re/im, x fastest):
 *   spinor  [n_rhs][t][z][y][x][spin 4][colour 3]   over the dynamical time
 *           slices only (T-1 of them for SF, T otherwise);
 *   links   [mu 4][x0][z][y][x][3][3]   over T+1 stored slices for SF (so the
 *           fixed boundary links are representable), T otherwise;
 *   force   same shape as the links: the Hermitian traceless matrix
 *           G_mu(n) = sum_a F^a_mu(n) T^a, T^a = lambda^a/2, where
 *           F^a = dS/dw^a under U_mu(n) -> exp(i w T^a) U_mu(n).  Links that
 *           never enter D hold exactly 0.
 *
 * Ownership: every *_dev pointer is device memory owned by the caller (for
 * example a torch tensor); the library never frees it.  The handle owns its
 * packed copies of the links, its workspaces and solver state.
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  mfq_dslash is
 * asynchronous on it.  The solves and the force are host-blocking on return
 * (convergence is data dependent and the statistics are host outputs); all
 * their device work is ordered on `stream`.
 *
 * Errors: functions return an mfq_status.  Negative values are hard errors;
 * mfq_last_error() then returns a message (thread local).  MFQ_NOT_CONVERGED
 * still writes the best solution and per-RHS statistics.  Nothing aborts or
 * throws across this boundary.  One handle must not be used by two threads at
 * the same time.
 */
#ifndef MFQ_H
#define MFQ_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mfq_handle mfq_handle;

typedef enum {
  MFQ_OK = 0,
  MFQ_NOT_CONVERGED = 1, /* max_iter reached; best x and stats written       */
  MFQ_FELL_BACK = 2,     /* learned preconditioner stagnated: CG finished it */
  MFQ_ERR_ARG = -1,      /* invalid argument or non-finite input             */
  MFQ_ERR_HIP = -2,      /* a HIP runtime call failed                        */
  MFQ_ERR_NOMEM = -3,    /* device allocation failed                         */
  MFQ_ERR_STATE = -4     /* call not valid in the handle's state             */
} mfq_status;

typedef enum { MFQ_BC_SF = 0, MFQ_BC_PERIODIC = 1, MFQ_BC_ANTIPERIODIC_T = 2 } mfq_bc;

/* Precision of the inner CG iteration.  All forms keep the solution and the
 * true residual in FP64 and reduce every dot product in FP64.
 *   FP64            plain FP64 CG.
 *   FP32_RELIABLE   FP32 vectors and links; FP64 reliable updates (the true
 *                   residual b - A x is recomputed in FP64 whenever the inner
 *                   residual has dropped by reliable_delta, and the FP32
 *                   recursion continues from it).
 *   FP16_REFINE     FP16 vectors (per-site FP32 norm) and FP16 links, FP32
 *                   arithmetic, FP32 solution correction; FP64 defect
 *                   correction (restart from the FP64 true residual).
 * This is the mixed-precision (flexible) inner/outer split of Section 3.2,
 * done on one GPU with the outer FP64 steps on the device. */
typedef enum { MFQ_PREC_FP64 = 0, MFQ_PREC_FP32_RELIABLE = 1, MFQ_PREC_FP16_REFINE = 2 } mfq_prec;

/* Operators for mfq_dslash (H is the hopping term, D = 1 - kappa H):
 *   HOP_EO   out_even = H_eo in_odd,  out_odd = 0
 *   HOP_OE   out_odd  = H_oe in_even, out_even = 0
 *   HOP      out = H in     (both parities)      HOP_DAG  out = H^+ in
 *   D, DDAG, DDAGD          out = D in, D^+ in, D^+ D in
 *   SCHUR, SCHUR_DAG, SCHUR_NORMAL   out_even = D^ in_even, D^^+ in_even,
 *            D^^+ D^ in_even with D^ = 1 - kappa^2 H_eo H_oe, the Schur
 *            complement of the even/odd blocks of D (the site even/odd
 *            preconditioning of Sec. 3.1); out_odd = 0, in_odd is ignored  */
typedef enum {
  MFQ_OP_HOP_EO = 0,
  MFQ_OP_HOP_OE = 1,
  MFQ_OP_D = 2,
  MFQ_OP_DDAG = 3,
  MFQ_OP_DDAGD = 4,
  MFQ_OP_HOP = 5,
  MFQ_OP_HOP_DAG = 6,
  MFQ_OP_SCHUR = 7,
  MFQ_OP_SCHUR_DAG = 8,
  MFQ_OP_SCHUR_NORMAL = 9
} mfq_op;

/* Solve route for CG (precond MFQ_PC_NONE):
 *   FULL   CG on the normal operator D^+D over every site (x = (D^+D)^-1 b;
 *          the force takes one such solve: Z = (D^+D)^-1 g5 Phi).
 *   SCHUR  even/odd preconditioned: every solve of D (or D^+) runs CG on
 *          D^^+ D^ over the even sites (half the volume, better conditioned)
 *          and rebuilds the odd sites; (D^+D)^-1 b then takes two of them
 *          (D^+ w = b, D x = w) and the force too (D X = Phi, D^+ Y = X).
 *          tol applies to each Schur solve's own normal equations; the
 *          statistics report the summed iterations and the final FP64
 *          residual of the full system. */
typedef enum { MFQ_ROUTE_FULL = 0, MFQ_ROUTE_SCHUR = 1 } mfq_route;

/* Solver selection: NONE is CG on D^+D; PTC is restarted flexible GMRES
 * (restart = mfq_solve_params.restart; prec FP64: the cycle in FP64, else
 * the basis, the operator inside the cycle and the network's input and
 * output in FP32, with FP64 dot-product sums, solution and true-residual
 * restarts) right-preconditioned by
 * the learned parallel-transport network, with CG as the fallback when a
 * cycle stagnates or breaks down (status MFQ_FELL_BACK); IDENTITY is the same
 * GMRES without preconditioner (the reference the network is measured
 * against).  FGMRES keeps its basis (restart + 1 fields of n_rhs RHS, plus
 * restart directions with PTC, in the cycle's precision) in the handle
 * between calls, freed by mfq_destroy; with use_graph one restart cycle is
 * captured once and replayed.  BLOCKCG is block conjugate gradients on D^+D: the n_rhs (<= 8)
 * right-hand sides share one Krylov space (the CG counterpart of the block
 * Krylov solvers of Sec. 3.1); FP64 only (prec must be MFQ_PREC_FP64, else
 * MFQ_ERR_ARG), every iteration is one D^+D on all RHS plus n x n complex
 * Gram matrices and solves in FP64; it restarts from the FP64 true residual
 * if the recursive residual drifted, and hands the remaining residual to
 * batched CG (status MFQ_FELL_BACK) if an n x n solve breaks down. */
typedef enum {
  MFQ_PC_NONE = 0,
  MFQ_PC_PTC = 1,
  MFQ_PC_IDENTITY = 2,
  MFQ_PC_BLOCKCG = 3,
  MFQ_PC_BICGSTAB = 4,
  MFQ_PC_GL_BICGSTAB = 5,
  MFQ_PC_BL_BICGSTAB = 6
} mfq_pc;
/* The paper's own solvers (Sec. 3.1-3.2), selected by BICGSTAB (BiCGStab
 * per RHS, the sequential baseline), GL_BICGSTAB (Global BiCGStab: Frobenius
 * inner products over the block) and BL_BICGSTAB (Block BiCGStab: n x n
 * alpha and beta from the shadow block), n_rhs <= 8: they solve D (and D^+)
 * itself, not the normal equations, through the even/odd Schur complement
 * D^ = 1 - kappa^2 H_eo H_oe (odd sites rebuilt).  prec FP64: FP64
 * throughout; FP32_RELIABLE: FP64 outer iteration whose right preconditioner
 * is an FP32 BiCGStab solve per RHS to the relative tolerance inner_tol (at
 * most inner_max_iter iterations), the mixed-precision preconditioning of
 * Sec. 3.2; FP16 is refused.  The outer iteration stops on the FP64 true
 * residual |b_e - D^ x_e| <= tol |b_e| of the even system, restarting from
 * it (new shadow block) when the recursion lied or broke down (at most 5
 * restarts).  (D^+D)^-1 b takes two such solves (D^+ w = b, D x = w), the
 * force the two of Alg. 2 (D X = Phi, D^+ Y = X), mfq_solve_dirac one. */

typedef struct {
  int dims[4]; /* Lx, Ly, Lz, T: even, >= 2 (T >= 4 for SF); volume at most
                  4.4e7 sites and (volume / 2) * max(Lx / 2, Ly, Lz) < 2^31 */
  int bc;      /* mfq_bc                                                       */
  double kappa;/* 0 < kappa < 0.25                                             */
} mfq_lattice;

typedef struct {
  double tol;            /* per-RHS true relative residual |b - A x|/|b|     */
  int max_iter;          /* inner iterations per RHS before NOT_CONVERGED    */
  int prec;              /* mfq_prec                                          */
  double reliable_delta; /* reliable-update trigger (<= 0: default 0.1)      */
  int precond;           /* mfq_pc                                            */
  int restart;           /* FGMRES restart length (PTC / IDENTITY; <= 0: 16)  */
  int check_every;       /* iterations between host polls (<= 0: default)    */
  int use_graph;         /* capture the inner iterations in a hipGraph        */
  int route;             /* mfq_route (SCHUR needs precond MFQ_PC_NONE)       */
  double inner_tol;      /* BiCGStab solvers, prec FP32_RELIABLE: relative
                            tolerance of the inner FP32 solves (<= 0: 1e-4) */
  int inner_max_iter;    /* ... and their iteration cap (<= 0: 500)          */
} mfq_solve_params;

typedef struct {
  int iters;             /* inner iterations                                 */
  int reliable_updates;  /* FP64 true-residual evaluations                   */
  double true_rel_resid; /* final FP64 |b - A x| / |b|                        */
  double seconds;        /* wall time of the whole call                      */
  int status;            /* mfq_status of this RHS                            */
  int inner_iters;       /* BiCGStab with FP32 inner solves: inner iterations,
                            summed over the inner calls (else 0)             */
  int inner_calls;       /* ... and the number of inner calls                */
} mfq_solve_stats;

/* Create a handle for one lattice and pack the links (canonical FP64 device
 * array, see above) into the internal FP64, FP32 and FP16 copies.  The FP32
 * and FP16 copies store the first two rows of each link and rebuild the third
 * (unit determinant); if any link is not SU(3) to 1e-10 the handle still
 * works in FP64, while FP32/FP16 solves and the learned preconditioner
 * return MFQ_ERR_ARG. */
int mfq_create(const mfq_lattice* lat, const double* links_dev, void* stream, mfq_handle** out);

/* Repack the links after they changed (for example after an MD step). */
int mfq_update_links(mfq_handle* h, const double* links_dev, void* stream);

/* out = op(in) for n_rhs canonical spinors, computed in FP64.  Asynchronous. */
int mfq_dslash(mfq_handle* h, int op, const double* in_dev, double* out_dev, int n_rhs, void* stream);

/* mfq_dslash (FP64, every mfq_op) without any device allocation, for
 * callers that cannot allocate (code under stream capture, serving loops
 * that forbid hipMalloc).  The packed input, output and (for DDAGD) the
 * intermediate field live in a fixed 64 MiB per-device workspace inside the
 * library instead of the handle's workspaces; the handle's packed links are
 * used as they are.  Sizes: 2 (3 for DDAGD and the SCHUR ops) packed fields of
 * n_rhs * 2 * 12 * vs * 16 bytes, vs ~ (sites per parity rounded up to an odd
 * multiple of 16), must fit in 64 MiB, else MFQ_ERR_ARG and nothing is
 * written (for example an 8^3x8 SF lattice takes up to 18 RHS).  Results
 * equal mfq_dslash's to rounding.  Asynchronous on `stream`.  Every call on
 * one GPU shares that GPU's workspace: calls that overlap in time on one GPU
 * (different streams or threads) race and must be serialised by the caller. */
int mfq_dslash_noalloc(mfq_handle* h, int op, const double* in_dev, double* out_dev, int n_rhs, void* stream);

/* Same, with the storage/arithmetic precision of an inner solve (mfq_prec):
 * the input is rounded to that precision, the operator applied in it, and the
 * result widened back to FP64. */
int mfq_dslash_prec(mfq_handle* h, int op, int prec, const double* in_dev, double* out_dev, int n_rhs,
                    void* stream);

/* x_i = (D^+ D)^-1 b_i for i < n_rhs, all RHS in one batched CG (Section 3.1:
 * the blocked form of the linear equations); with params->route = SCHUR as
 * two even/odd-preconditioned solves (D^+ w = b, then D x = w).
 * stats_host: n_rhs records. */
int mfq_solve_multi_rhs(mfq_handle* h, const double* b_dev, double* x_dev, int n_rhs,
                        const mfq_solve_params* params, mfq_solve_stats* stats_host, void* stream);

/* x_i = D^-1 b_i (dagger 0) or (D^+)^-1 b_i (dagger 1): one line of Alg. 2
 * (its second line is D X = Phi, its third D^+ Y = X), through the even/odd
 * Schur complement: with precond NONE by CG on D^^+ D^ (route SCHUR), with
 * the BiCGStab selections by the paper's solvers.  Other selections return
 * MFQ_ERR_ARG.  stats_host: n_rhs records (true_rel_resid: of the even
 * system). */
int mfq_solve_dirac(mfq_handle* h, int dagger, const double* b_dev, double* x_dev, int n_rhs,
                    const mfq_solve_params* params, mfq_solve_stats* stats_host, void* stream);

/* Alg. 2 for n_rhs pseudo-fermions: one batched normal-equation solve
 * Z = (D^+ D)^-1 g5 Phi gives Y = (D^+)^-1 D^-1 Phi = g5 Z and X = D^-1 Phi =
 * D^+ Y (route FULL), or the two solves of Alg. 2 themselves, D X = Phi and
 * D^+ Y = X, each through the even/odd Schur complement (route SCHUR); then
 * force_dev (links shape) = sum_i f[x_i, y_i] (Eq. 3) and action_host[i] =
 * |x_i|^2 (Eq. 2).  x_dev / y_dev may be NULL; if given they receive X and Y
 * (spinor shape).  The statistics of route SCHUR sum both solves'
 * iterations; true_rel_resid is that of the last solve's normal equations. */
int mfq_fermion_force(mfq_handle* h, const double* phi_dev, int n_rhs, const mfq_solve_params* params,
                      double* force_dev, double* action_host, double* x_dev, double* y_dev,
                      mfq_solve_stats* stats_host, void* stream);

/* The even/odd-preconditioned action variant S = sum_i |D^-1 phi_i,e|^2
 * (phi on the even sites; the odd sites of phi_dev are ignored), the form an
 * HMC with even/odd preconditioning integrates (Sec. 3.1).  One CG on
 * D^^+ D^ over the even sites gives Y_e = g5 (D^^+ D^)^-1 g5 phi_e and
 * X_e = D^^+ Y_e = D^-1 phi_e; with X_o = kappa H_oe X_e and
 * Y_o = kappa (H^+)_oe Y_e the force of this action is the Eq. 3 force of the
 * full-lattice X and Y, so force_dev is filled as by mfq_fermion_force;
 * action_host[i] = |X_e,i|^2.  x_dev / y_dev (may be NULL) receive the full X
 * and Y.  params->route is ignored (always the even-site CG). */
int mfq_fermion_force_eo(mfq_handle* h, const double* phi_dev, int n_rhs, const mfq_solve_params* params,
                         double* force_dev, double* action_host, double* x_dev, double* y_dev,
                         mfq_solve_stats* stats_host, void* stream);

/* ---- molecular dynamics: the HMC of Sec. 2 on the GPU -------------------
 * Momenta use the force's layout: per link the Hermitian traceless
 * P_mu(n) = sum_a P^a T^a (canonical links shape, FP64).  Equations of
 * motion dU/dt = i P U, dP/dt = -G with G from mfq_fermion_force; the
 * Hamiltonian H = 1/2 sum P^a P^a + sum_i |D^-1 phi_i|^2 (pseudo-fermion
 * action only; the gauge action is not part of this library).  Only links
 * that enter D move; the others (SF: spatial links at x0 = 0 and T, temporal
 * links at x0 = 0, T-1, T) keep their values, and their momenta are ignored. */

/* out_host = 1/2 sum_a P^a P^a = sum over entering links of Tr P^2 (FP64,
 * fixed-order reduction on the device).  Host-blocking. */
int mfq_kinetic_energy(mfq_handle* h, const double* mom_dev, double* out_host, void* stream);

/* mom_dev <- mom_dev - eps * force_dev on the entering links.  Asynchronous. */
int mfq_md_momenta(mfq_handle* h, const double* force_dev, double* mom_dev, double eps, void* stream);

/* links_dev <- exp(i eps P) links_dev on the entering links (3x3 exponential
 * in FP64: scaling and squaring of a degree-12 Taylor polynomial), then the
 * handle's packed copies are refreshed (as mfq_update_links).  Host-blocking. */
int mfq_md_links(mfq_handle* h, const double* mom_dev, double* links_dev, double eps, void* stream);

typedef struct {
  double tau;          /* trajectory length (> 0)                               */
  int n_steps;         /* leapfrog steps (>= 1), dt = tau / n_steps             */
  double rand_uniform; /* the Metropolis draw in [0, 1), supplied by the caller  */
} mfq_hmc_params;

typedef struct {
  double delta_h;                  /* H_new - H_old, FP64                       */
  double kinetic_old, kinetic_new; /* 1/2 sum P^a P^a                           */
  double action_old, action_new;   /* sum_i |D^-1 phi_i|^2                      */
  int accepted;                    /* 1 if rand_uniform < exp(-delta_h), i.e.
                                      log(rand_uniform) < -delta_h            */
  int force_evals;                 /* n_steps + 1                               */
  int solver_iters;                /* summed over force evaluations and RHS      */
  double seconds;
} mfq_hmc_result;

/* One HMC trajectory with the leapfrog integrator (P -= dt/2 G; then n_steps
 * times U <- exp(i dt P) U, G(U), P -= dt G, the last kick dt/2), every force
 * from mfq_fermion_force with `sp` (so route, precision and solver are the
 * caller's choice), Delta H in FP64 and the Metropolis decision with the
 * caller's draw.  On acceptance links_dev / mom_dev hold the new U and P; on
 * rejection they are restored to their values on entry (and the handle's
 * packed links with them).  phi_dev: n_rhs canonical pseudo-fermions, fixed
 * during the trajectory.  Returns the worst solver status (MFQ_OK,
 * MFQ_NOT_CONVERGED, MFQ_FELL_BACK) or a negative error.  Host-blocking. */
int mfq_hmc_trajectory(mfq_handle* h, double* links_dev, double* mom_dev, const double* phi_dev, int n_rhs,
                       const mfq_hmc_params* hp, const mfq_solve_params* sp, mfq_hmc_result* out, void* stream);

/* ---- many lattices in one persistent launch per CG phase --------------
 * A batch groups distinct handles (lattices of any size, each with its own
 * links and kappa) with n_rhs[i] right-hand sides each (1..64).  Every CG
 * phase of all lattices runs as one launch of a persistent kernel over a
 * static list of (lattice, site tile, RHS group) tiles; the iterations are
 * captured in a hipGraph.  Each lattice keeps its own per-RHS scalars and
 * convergence; precision is fixed per batch (mfq_prec).  The batch uses the
 * handles' workspaces: using a handle elsewhere with more RHS reallocates
 * them, after which mfq_batch_solve returns MFQ_ERR_STATE (re-create it).
 * Destroy the batch before its handles. */
typedef struct mfq_batch mfq_batch;

int mfq_batch_create(mfq_handle** hs, int n_lat, const int* n_rhs, int prec, void* stream, mfq_batch** out);

/* b_dev[i], x_dev[i]: canonical spinors of lattice i (n_rhs[i] each).
 * stats_host: sum of n_rhs records, lattice by lattice.  Host-blocking. */
int mfq_batch_solve(mfq_batch* batch, const double* const* b_dev, double* const* x_dev,
                    const mfq_solve_params* params, mfq_solve_stats* stats_host, void* stream);

/* One-shot form: create, solve, destroy. */
int mfq_solve_batch(mfq_handle** hs, int n_lat, const double* const* b_dev, double* const* x_dev,
                    const int* n_rhs, const mfq_solve_params* params, mfq_solve_stats* stats_host,
                    void* stream);

/* Persistent grid size chosen by the batch's autotuning (workgroups). */
int mfq_batch_grid(mfq_batch* batch);

/* Whether the inner hopping phases split each site's four directions over
 * wavefronts (1) or run one thread per site (0), as chosen by the tuning. */
int mfq_batch_split(mfq_batch* batch);

/* Override the tuned launch shape of the persistent kernels: grid size
 * (workgroups, 1..65536) and the direction split (0 or 1); drops the
 * captured graphs. */
int mfq_batch_set_shape(mfq_batch* batch, int grid, int split);

void mfq_batch_destroy(mfq_batch* batch);

/* ---- learned preconditioner: gauge-covariant parallel-transport network --
 * M = L2 L1 with L(psi)[c'](n) = sum_c sum_p W[p][c'][c] (T_p psi[c])(n) over
 * the 9 paths p (identity; U_mu(n) psi(n+mu); U_mu(n-mu)^+ psi(n-mu)), W a
 * complex 4x4 spin matrix, channels 1 -> 8 -> 1, linear.  Weights are
 * 2 x 9 x 8 x 16 complex numbers, passed as interleaved FP64 re/im:
 * W1[p][c'][s'][s] (layer 1), then W2[p][c][s'][s] (layer 2).  Training keeps
 * FP32 master weights; inference uses their BF16-rounded values with FP32
 * accumulation.  The network is trained on the GPU by this library's forward,
 * backward and Adam kernels, on pairs (r_k, e_k) that CG generates.
 * Pair arrays hold n_pairs canonical spinors (one RHS each). */

/* Random initial weights (identity path near 1/sqrt(8) in both layers). */
int mfq_precond_init(mfq_handle* h, unsigned long long seed, double scale);
int mfq_precond_set_weights(mfq_handle* h, const double* w_host);
/* which = 0: FP32 master weights, 1: BF16-rounded inference weights,
 * 2 / 3: Adam's first / second moment estimates (same layout: the real part
 * holds the moment of Re W, the imaginary part that of Im W). */
int mfq_precond_get_weights(mfq_handle* h, int which, double* w_host);
/* out = M in for n_rhs canonical spinors (inference weights). */
int mfq_precond_apply(mfq_handle* h, const double* in_dev, double* out_dev, int n_rhs, void* stream);
/* loss = mean_k |M r_k - e_k|^2 / |e_k|^2 at the master weights and its
 * gradient (dL/dRe W + i dL/dIm W, same layout as the weights). */
int mfq_precond_loss_grad(mfq_handle* h, const double* r_dev, const double* e_dev, int n_pairs, double* loss_host,
                          double* grad_host, void* stream);
/* `steps` full-batch Adam steps (beta = 0.9, 0.999); loss before each step in
 * loss_hist_host[steps] (may be NULL). */
int mfq_precond_train(mfq_handle* h, const double* r_dev, const double* e_dev, int n_pairs, int steps, double lr,
                      double* loss_hist_host, void* stream);
/* Training pairs from plain FP64 CG with a known solution: for the n_rhs
 * canonical spinors xi (device, FP64) CG runs on b = A xi from x_0 = 0, and
 * for j = 0..n_snap-1 its iterate x_k after k = every * j iterations gives
 * r = (b - A x_k) / |b - A x_k| and e = (xi - x_k) / |b - A x_k|, so that
 * A e = r.  The pair at k = 0 is (A xi, xi) / |A xi|: its error is spread
 * over the whole spectrum, the later ones lean to the low modes.  r_out,
 * e_out: n_snap * n_rhs canonical spinors each (device), pair j-major.
 * xi must be nonzero and finite (MFQ_ERR_ARG otherwise). */
int mfq_precond_pairs(mfq_handle* h, const double* xi_dev, int n_rhs, int every, int n_snap, double* r_out,
                      double* e_out, void* stream);
int mfq_precond_save(mfq_handle* h, const char* path);
int mfq_precond_load(mfq_handle* h, const char* path);

/* Thread-local message for the last negative status. */
const char* mfq_last_error(void);

/* Average device time (ms) of one launch of the dominant solver kernel (the
 * fused half-dslash of the inner CG at precision `prec` for n_rhs RHS, both
 * parities, in the solver's launch shape), timed with HIP events around
 * `iters` back-to-back launches on `stream`, on a fixed nonzero field. */
int mfq_time_hop(mfq_handle* h, int prec, int n_rhs, int iters, void* stream, double* ms_out);

/* Launch-shape autotuning of the inner solver's hopping kernel (on by
 * default).  The first solve (or mfq_time_hop) for a given (n_rhs, precision)
 * times candidate (sites per workgroup, RHS per workgroup, tile order) shapes
 * with HIP events and keeps the fastest; MFQ_AUTOTUNE_CACHE, if set, names a
 * text file where choices are stored and looked up; if it is not set, the
 * table tune_gfx950.txt next to the library (shapes tuned on MI355X for the
 * shipped workloads) is looked up and nothing is written.  Turning it off uses a
 * fixed default shape.  Changing the setting drops tuned shapes and graphs. */
int mfq_set_autotune(mfq_handle* h, int on);

/* The shape the inner solver uses for (precision, n_rhs): shape5 (host, 5
 * ints) receives {sites per workgroup, RHS per workgroup, tile order flags
 * (bit 0: each XCD walks a contiguous chunk of tiles; bit 1: tiles walked
 * (z, t) plane by plane over blocks of consecutive z, t before z; bit 2: the
 * workgroup's links staged in an LDS tile shared by its RHS rows),
 * time-sweep length (0: one site per thread; else each thread walks that many
 * time slices of one spatial site, sites per workgroup then counting spatial
 * sites), direction split (0, or 2 / 4 wavefronts sharing the 4 directions of
 * 64 sites of one RHS)}. */
int mfq_hop_shape(mfq_handle* h, int prec, int n_rhs, int* shape5);

void mfq_destroy(mfq_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* MFQ_H */
