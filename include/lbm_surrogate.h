/*
 * lbm_surrogate.h -- C ABI of the learned warm start: BF16 MFMA kernels for a
 * 3-D convolutional encoder-decoder that maps an obstacle mask and a body
 * force to the steady (rho, u) field of the lattice Boltzmann channel, plus
 * the training pieces (loss, Adam) and the conversions to and from the
 * lattice fields.  Not part of the paper: the paper's solver (Sec. 2.1)
 * produces the training data and judges every prediction, because a
 * prediction only sets the initial state of lbm_set_equilibrium and the
 * solver then runs to its own steady state.
 *
 * Tensors are channels-last BF16 (bit pattern in uint16): element
 * (n, d, h, w, c) sits at ptr[(((n*D + d)*H + h)*W + w)*ldc + c].  ldc >= C
 * lets a tensor be a channel slice of a wider buffer (skip concatenation
 * without copies).  C and ldc must be multiples of 8 and ptr 16-byte aligned.
 * Convolutions are 3x3x3 (padding 1, stride 1 or 2) or 1x1x1 (padding 0,
 * stride 1).  Weights of a layer with Cin inputs, Cout outputs and T taps
 * (27 or 1) are stored "K-major": w[co][t*Cin + ci], with K = T*Cin rounded up
 * to a multiple of 32 (the padding is zero).  All arithmetic accumulates in
 * FP32.  Every call enqueues on `stream` (hipStream_t, NULL = null stream),
 * allocates nothing and returns lbm_status (LBM_EINVAL on bad shapes).
 */
#ifndef LBM_SURROGATE_H_
#define LBM_SURROGATE_H_

#include <stdint.h>

#include "lbm.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  void* ptr;                 /* device pointer to element (0,0,0,0,0) */
  int32_t n, d, h, w, c;     /* batch, depth (z), height (y), width (x), channels */
  int32_t ldc;               /* channel stride in elements */
} lbm_tensor5;

/* K-major row length of a weight with `taps` taps and `cin` inputs. */
int32_t lbm_conv_kpad(int32_t taps, int32_t cin);

/* y = act(conv(x, w) + bias).  ksize 3 (pad 1) or 1 (pad 0); stride 1 or 2
 * (output size ceil(in/stride)).  relu = 1 applies max(0, .).  bias: FP32
 * [Cout] device pointer or NULL. */
lbm_status lbm_conv3d_fwd(const lbm_tensor5* x, const uint16_t* w, const float* bias, const lbm_tensor5* y,
                          int32_t ksize, int32_t stride, int32_t relu, void* stream);

/* Gradient with respect to the input.  w_t is the transposed weight made by
 * lbm_conv3d_weight_t (layout wt[ci][t*Cout + co]).  If `act` is non-NULL the
 * result is multiplied by (act > 0): the ReLU derivative of the layer that
 * produced x, whose output `act` is.  accumulate = 1 adds into dx. */
lbm_status lbm_conv3d_bwd_data(const lbm_tensor5* dy, const uint16_t* w_t, const lbm_tensor5* dx,
                               const lbm_tensor5* act, int32_t ksize, int32_t stride, int32_t accumulate,
                               void* stream);

/* Gradient with respect to the weights and bias, ADDED (FP32 atomics) into
 * dw[co][kpad] and dbias[Cout] (dbias may be NULL).  Clear them first.  The
 * summation order of the atomics varies from run to run, so results agree
 * to FP32 rounding, not bit for bit.  LBM_EINVAL if dbias is given with
 * Cout > 2048. */
lbm_status lbm_conv3d_bwd_weight(const lbm_tensor5* x, const lbm_tensor5* dy, float* dw, float* dbias,
                                 int32_t ksize, int32_t stride, void* stream);

/* Transposed weight for lbm_conv3d_bwd_data: wt[ci][t*Cout + co] (padded to
 * lbm_conv_kpad(taps, cout)) from w[co][t*Cin + ci]; FP32 master -> BF16. */
lbm_status lbm_conv3d_weight_t(const float* w_master, int32_t taps, int32_t cin, int32_t cout,
                               uint16_t* w_bf16, uint16_t* wt_bf16, void* stream);

/* Nearest-neighbour 2x upsampling of x into y (y dims = 2 x dims) and its
 * adjoint (dx = sum of the 8 children of dy; accumulate adds into dx). */
lbm_status lbm_upsample2(const lbm_tensor5* x, const lbm_tensor5* y, void* stream);
lbm_status lbm_upsample2_bwd(const lbm_tensor5* dy, const lbm_tensor5* dx, int32_t accumulate, void* stream);

/* Masked mean-squared error over the first `nch` channels of pred against an
 * FP32 target [voxels][nch]; voxels with weight 0 are skipped.  Adds the loss
 * into *loss (device FP32) and writes dpred = 2 (pred - target)/count (BF16,
 * channels >= nch set to 0). */
lbm_status lbm_mse_loss(const lbm_tensor5* pred, const float* target, const uint8_t* weight, int32_t nch,
                        float inv_count, const lbm_tensor5* dpred, float* loss, void* stream);

/* Adam on FP32 master weights (bias-corrected, step t >= 1). */
lbm_status lbm_adam_step(float* w, const float* g, float* m, float* v, int64_t n, float lr, float beta1,
                         float beta2, float eps, int32_t t, void* stream);

/* Network input of one sample: channels (solid, normalised force, wall-normal
 * coordinate, 0...) from a device solid mask [D][H][W] (uint8) and the force
 * g_x; x has c = 8. */
lbm_status lbm_surrogate_input(const uint8_t* solid, double gx, const lbm_tensor5* x, void* stream);

/* Training target of one sample from lattice fields (device FP64 rho[V],
 * u[3][V]): t[v] = (u_x, u_y, u_z, rho - rho0) / (gx * scale), FP32 [V][4];
 * weight[v] = 1 for fluid cells, 0 for solid cells. */
lbm_status lbm_surrogate_target(const double* rho, const double* u, const uint8_t* solid, double rho0, double gx,
                                double scale, int64_t voxels, float* target, uint8_t* weight, void* stream);

/* Inverse of lbm_surrogate_target applied to a prediction pred[v][0..3]
 * (BF16): rho, u (FP64 device) for lbm_set_equilibrium; solid cells rho0, 0. */
lbm_status lbm_surrogate_fields(const lbm_tensor5* pred, const uint8_t* solid, double rho0, double gx,
                                double scale, double* rho, double* u, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* LBM_SURROGATE_H_ */
