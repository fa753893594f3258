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

// out = scale_out * L2(L1(scale_in * in)), hid: 8 channels x n_rhs (FP32).
template <typename SI, typename SO>
hipError_t ptc_forward(const Geom& g, Links<float> L, Field<SI> in, Field<float> hid, Field<SO> out, const f2* W1,
                       const f2* W2, int n_rhs, float in_scale, float out_scale, hipStream_t st);

// The same forward pass with both mixings on the BF16 matrix instruction
// (inference): chi (ptc_chi_floats FP32 values) holds the layer-2 mixings
// chi_p before transport, ops (ptc_ops_bytes) the weight operands that
// ptc_pack_ops lays out from the inference weights.
size_t ptc_ops_bytes();
size_t ptc_chi_floats(const Geom& g, int n_rhs);
hipError_t ptc_pack_ops(const f2* W1, const f2* W2, void* ops, hipStream_t st);
template <typename SI, typename SO>
hipError_t ptc_forward_mx(const Geom& g, Links<float> L, Field<SI> in, float* chi, Field<SO> out, const void* ops,
                          int n_rhs, hipStream_t st);

// gh[k*8 + c] = sum_p W2[p][c]^+ (T_pbar gy_k): the adjoint of layer 2.
hipError_t ptc_adjoint2(const Geom& g, Links<float> L, Field<float> gy, Field<float> gh, const f2* W2, int n_pairs,
                        hipStream_t st);

// grad[p][co][ci][16] = sum over sites, colours, pairs of g[co] (T_p x[ci])^+
// (partials per workgroup in `part`, reduced in fixed order into grad, FP64).
template <typename SX>
hipError_t ptc_weight_grad(const Geom& g, Links<float> L, Field<SX> x, int c_in, Field<float> gf, int c_out,
                           int n_pairs, double* part, double* grad, hipStream_t st);

// diff = y - e; gy = 2 diff / (n |e|^2); loss partials |diff|^2 / |e|^2.
hipError_t ptc_loss_grad_out(const Geom& g, Field<float> y, Field<double> e, const double* enorm2, Field<float> gy,
                             int n_pairs, double* part, hipStream_t st);

// Adam on the FP32 master weights (Re and Im as separate parameters);
// also refreshes the BF16-rounded inference copy.
hipError_t ptc_adam(float* w, const double* grad, float* m, float* v, int n_real, int t, double lr, double b1,
                    double b2, double eps, f2* w_infer, hipStream_t st);

}  // namespace mfq
