// Parallel-transport convolution network (learned preconditioner): sizes and
// kernel launchers.
#pragma once

#include "internal.h"

namespace mfq {

constexpr int PTC_PATHS = 9;
constexpr int PTC_HIDDEN = 8;
// complex weights: W1[p][c'][16] (1 -> 8) and W2[p][c][16] (8 -> 1)
constexpr int PTC_W1 = PTC_PATHS * PTC_HIDDEN * 16;
constexpr int PTC_W2 = PTC_PATHS * PTC_HIDDEN * 16;
constexpr int PTC_NW = PTC_W1 + PTC_W2;

// The forward pass out = L2(L1(in)) with both channel mixings on the BF16
// matrix instruction (inference): chi (ptc_chi_floats FP32 values) holds
// the layer-2 mixings chi_p before transport, ops (ptc_ops_bytes) the weight
// operands that ptc_pack_ops lays out from the inference weights.
size_t ptc_ops_bytes();
size_t ptc_chi_floats(const Geom& g, int n_rhs);
hipError_t ptc_pack_ops(const f2* W1, const f2* W2, void* ops, hipStream_t st);
template <typename SI, typename SO>
hipError_t ptc_forward_mx(const Geom& g, Links<float> L, Field<SI> in, float* chi, Field<SO> out, const void* ops,
                          int n_rhs, hipStream_t st);

// Training on the matrix instruction with FP32 weights: ptc_pack_ops_split
// lays out hi and lo BF16 operand sets (2 * ptc_ops_bytes()); the forward
// pass also stores layer 1's result in hid; ptc_adj_weights forms the
// layer-1-shaped weights Wa[q][c] = W2[qbar][c]^+ (PTC_W1 complex), with which
// ptc_adjoint2_mx computes gh[k*8 + c] = sum_q Wa[q][c] (T_q gy_k).
hipError_t ptc_pack_ops_split(const f2* W1, const f2* W2, void* ops, hipStream_t st);
hipError_t ptc_adj_weights(const f2* W2, f2* Wa, hipStream_t st);
hipError_t ptc_forward_mx_train(const Geom& g, Links<float> L, Field<double> in, float* chi, Field<float> hid,
                                Field<float> out, const void* ops_split, int n_rhs, hipStream_t st);
hipError_t ptc_adjoint2_mx(const Geom& g, Links<float> L, Field<float> gy, Field<float> gh, const void* ops_adj_split,
                           int n_pairs, hipStream_t st);

// The weight gradients grad[p][co][ci][16] = sum over pairs, sites and
// colours of g[co] (T_p x[ci])^+, on the BF16 matrix instruction: LAYER 1
// with x = the input pairs (c_in = 1) and gf = the hidden-layer gradient (8
// channels), into grad[W1]; LAYER 2 with x = the hidden field (8 channels)
// and gf = the output gradient (1 channel), into grad[W2] (as
// sum (T_pbar g) x^+).  nblk workgroups
// each store a partial C (ptc_wgrad_mx_part_floats(nblk) floats in part).
size_t ptc_wgrad_mx_part_floats(int nblk);
template <int LAYER, typename SX>
hipError_t ptc_weight_grad_mx(const Geom& g, Links<float> L, Field<SX> x, Field<float> gf, int n_pairs, int nblk,
                              float* part, double* grad, hipStream_t st);

// diff = y - e; gy = 2 diff / (n |e|^2); loss partials |diff|^2 / |e|^2.
hipError_t ptc_loss_grad_out(const Geom& g, Field<float> y, Field<double> e, const double* enorm2, Field<float> gy,
                             int n_pairs, double* part, hipStream_t st);

// Adam on the FP32 master weights (Re and Im as separate parameters);
// also refreshes the BF16-rounded inference copy.
hipError_t ptc_adam(float* w, const double* grad, float* m, float* v, int n_real, int t, double lr, double b1,
                    double b2, double eps, f2* w_infer, hipStream_t st);

}  // namespace mfq
