/*
 * mri_surrogate.h -- learned fast-stage surrogate of libmri.  The stage solve
 * of the MRI algorithm (Sec. 2.1 step 2b: the modified fast IVP over one slow
 * stage) is taken in three parts:
 *   1. a coarse FP64 solve of the stage with few substeps (and the same with
 *      half as many, for a Richardson extrapolation);
 *   2. a small MLP, run with BF16 MFMA kernels (FP32 accumulation), predicts
 *      the correction from the coarse result to the plain FP64 stage with the
 *      workload's substeps, from the stage start state, the forcing and the
 *      stage length;
 *   3. a residual check on FP64 data compares the corrected state with the
 *      Richardson extrapolation of the two coarse solves and checks the
 *      mass-sum invariant; every cell that fails it, or that a coarse solve
 *      flagged, is integrated by the plain FP64 fast stage instead.
 * The paper has no surrogate; it is an addition to the method, and the plain
 * FP64 solve stays the reference for every result.
 *
 * Network (fixed for inference): 89 inputs -- log max(Y_k, 1e-30) for 21
 * species, T, the 3 forcing-polynomial coefficients of each of the 22 state
 * components (zero where the coupling table has fewer terms), log L (stage
 * length) -- standardized with training-set statistics; 3 hidden layers of
 * 256 with SiLU; 22 outputs = standardized corrections: for a species
 * log(Y_fine + 1e-8) - log(Y_base + 1e-8) (negative values clamped at 0), so
 * that an output error is a relative error of Y + 1e-8 (the floor of the error
 * metric); for T the plain difference T_fine - T_base.
 *
 * Conventions follow mri.h: device arrays are caller-owned; handles own their
 * device copies; invalid arguments return MRI_EINVAL before device work.
 * Bfloat16 arrays are passed as uint16_t bit patterns.
 */
#ifndef MRI_SURROGATE_H
#define MRI_SURROGATE_H

#include <stddef.h>
#include <stdint.h>

#include "mri.h"

#ifdef __cplusplus
extern "C" {
#endif

#define MRI_MLP_FEATURES 89      /* raw input features                      */
#define MRI_MLP_KPAD 96          /* padded input width of the first layer   */
#define MRI_MLP_OUTPUTS 22       /* corrections of the 22 components        */
#define MRI_MLP_STATS (2 * 89 + 3 * 22)
/* stats layout (FP64): x_mean[89], x_inv_std[89], y_mean[22], y_inv_std[22],
   y_std[22] (inverse std 1 where a feature is constant); y_* describe the
   corrections defined above. */

typedef struct mri_mlp mri_mlp;

/* ------------------------------------------------------------------------- */
/* Trainable MLP (training uses the same BF16 MFMA arithmetic as inference:   */
/* bf16 operands, FP32 accumulation, FP32 master weights and Adam state).     */
/* widths[0..n_layers]; params host FP32 packed W_1 [w1][w0], b_1 [w1], W_2,   */
/* b_2, ...; max_batch sizes the activation buffers.                          */
/* ------------------------------------------------------------------------- */
mri_status mri_mlp_create(int n_layers, const int *widths, const float *params, int max_batch,
                          mri_mlp **out);
void mri_mlp_destroy(mri_mlp *m);
int64_t mri_mlp_param_count(const mri_mlp *m);
/* Copies the FP32 master parameters / the last gradients (packed) to host. */
mri_status mri_mlp_get_params(const mri_mlp *m, float *params);
mri_status mri_mlp_get_grads(const mri_mlp *m, float *grads);
/* Forward pass of a batch.  X: device bf16 [batch][widths[0]]; Y (nullable):
   device f32 [batch][widths[L]].  Keeps the activations for the backward pass. */
mri_status mri_mlp_forward(mri_mlp *m, int batch, const uint16_t *X, float *Y,
                           mri_stream_t stream);
/* Backward pass of the last forward batch for the loss mean((Y - T)^2).
   T: device f32 [batch][widths[L]]; loss (nullable): device double, the batch
   loss is added to it.  Gradients are kept in the handle. */
mri_status mri_mlp_backward(mri_mlp *m, int batch, const float *T, double *loss,
                            mri_stream_t stream);
/* One Adam step on the kept gradients (bias-corrected, step count in the
   handle); refreshes the bf16 weight copies. */
mri_status mri_adam_step(mri_mlp *m, float lr, float beta1, float beta2, float eps,
                         mri_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Training data.  Stage samples are SoA with leading dimension ld:            */
/* Y0[c*ld + s] (c < 22) the stage start state, RHO[(p*22 + c)*ld + s]         */
/* (p < n_poly) the forcing coefficients, Lv[s] the stage length, Yb[c*ld + s] */
/* the base state the correction applies to (the coarse stage; NULL: Y0) and   */
/* Y1[c*ld + s] the plain FP64 stage result.                                   */
/* ------------------------------------------------------------------------- */
/* Feature / target statistics over n samples into stats (device FP64
   [MRI_MLP_STATS]): means and standard deviations from sums and sums of squares
   in a fixed reduction order (deterministic).  Allocates a partial-sum buffer
   and synchronizes the stream. */
mri_status mri_mlp_feature_stats(int64_t n, int64_t ld, const double *Y0, int n_poly,
                                 const double *RHO, const double *Lv, const double *Yb,
                                 const double *Y1, double *stats, mri_stream_t stream);
/* Standardized features X (device bf16 [batch][96], columns 89..95 zero) and
   targets T (nullable, device f32 [batch][22]) of the samples idx[0..batch)
   (idx NULL: 0..batch).  Species logarithms are taken in FP32, every other
   feature from its FP64 value; (raw - mean) * inv_std in FP64, rounded to FP32
   and then to bfloat16 (nearest even). */
mri_status mri_mlp_featurize(int batch, const int32_t *idx, int64_t ld, const double *Y0,
                             int n_poly, const double *RHO, const double *Lv, const double *Yb,
                             const double *Y1, const double *stats, uint16_t *X, float *T,
                             mri_stream_t stream);

/* ------------------------------------------------------------------------- */
/* Inference and the gated surrogate stage.                                  */
/* ------------------------------------------------------------------------- */
typedef struct mri_surrogate mri_surrogate;

/* Packs a trained MLP (host FP32 params, widths {89, 256, 256, 256, 22}, or
   {96, ...} as trained on the padded features of mri_mlp_featurize, whose
   padding columns are ignored) and its statistics (host FP64 [MRI_MLP_STATS])
   for the fused inference kernel. */
mri_status mri_surrogate_create(const int *widths, const float *params, const double *stats,
                                mri_surrogate **out);
void mri_surrogate_destroy(mri_surrogate *s);

/* One fused inference: the network reads the features of (y_in, rho, L) and
   its de-standardized output d is applied to `base` (NULL: y_in): y_out =
   (max(base, 0) + 1e-8) exp(d) - 1e-8 for a species, base + d for T.  y_in,
   base, y_out: device [22][ld]; rho: device [n_poly][22][ld], n_poly <= 3.
   y_out must not alias y_in or base. */
mri_status mri_surrogate_infer(const mri_surrogate *s, int n_cells, int ld, const double *y_in,
                               const double *base, double *y_out, int n_poly, const double *rho,
                               double L, mri_stream_t stream);

/* The residual check alone, on device arrays [22][ld]: v_coarse (coarse stage,
   n substeps), v_half (n/2 substeps), v_net (the network's correction of
   v_coarse).  With Ve = v_coarse + richardson (v_coarse - v_half), richardson =
   1 / (2^p - 1) for a fast method of order p,
     G = max(D, I),  D = max_c |v_net_c - Ve_c| / max(|Ve_c|, floor_c)
   (floor 1e-8 for mass fractions, 0 for T) and I = |sum_k (v_net_k - y_in_k) -
   L sum_p sum_k rho_(p,k) / (p + 1)| / sum_k |y_in_k| (the chemistry conserves
   sum_k Y_k, so over the stage the sum changes only by the integral of the
   forcing).  A cell is accepted when G <= gate_tol (never when G is NaN) and
   status_coarse (nullable, int32 [n_cells]) is 0; it gets y_out = v_net.
   Rejected cells are appended, in no particular order, to fallback_list
   (device int32 [n_cells]) and counted in *n_fallback (device).
   used_fallback (nullable, int32 [n_cells]): 1 for rejected cells;
   gate_value (nullable, FP64 [n_cells]): G. */
mri_status mri_surrogate_gate(int n_cells, int ld, const double *y_in, int n_poly,
                              const double *rho, double L, const double *v_coarse,
                              const double *v_half, const double *v_net,
                              const int32_t *status_coarse, double richardson, double gate_tol,
                              double *y_out, int32_t *used_fallback, double *gate_value,
                              int32_t *fallback_list, uint32_t *n_fallback, mri_stream_t stream);

mri_status mri_surrogate_workspace_bytes(int n_cells, int ld, int n_poly, size_t *bytes);

/* Gated surrogate stage over one stage of length L with forcing rho: the
   coarse FP64 stage (`coarse`: a fixed-step method, even n_sub >= 2; with
   coarse.stiff_limit > 0 its stiffness monitor flags, and so rejects, every
   cell with h B above the limit, h = L / n_sub) and the same with n_sub / 2, the network's correction of the coarse result, the
   residual check of mri_surrogate_gate (richardson from the coarse method's
   order; the correction and the check run in one launch and give bitwise the
   results of mri_surrogate_infer followed by mri_surrogate_gate), and the
   plain FP64 fast stage (`fallback` options) of every rejected cell,
   compacted, integrated and scattered back.  Nothing synchronizes the
   host: the fallback launch is sized for n_cells and its kernels stop at the
   count the check left on the device.  used_fallback (nullable, int32
   [n_cells]), gate_value (nullable, FP64 [n_cells]) as in mri_surrogate_gate;
   status_out (nullable, int32 [n_cells]): 0 for accepted cells, the fallback
   stage's MRI_CELL_* bits for the others; n_fallback (nullable, device
   uint32): the number of fallback cells.  ws: device workspace of
   mri_surrogate_workspace_bytes().  y_out may alias y_in. */
mri_status mri_surrogate_stage(const mri_surrogate *s, const mri_mech *mech,
                               const mri_fast_opts *coarse, const mri_fast_opts *fallback,
                               double gate_tol, int n_cells, int ld, const double *y_in,
                               double *y_out, int n_poly, const double *rho, double L,
                               int32_t *used_fallback, double *gate_value, int32_t *status_out,
                               uint32_t *n_fallback, void *ws, size_t ws_bytes,
                               mri_stream_t stream);

/* Forcing assembly of one slow stage as in mri_slow_step (Sec. 2.1 step 2a):
   rho[k] = (1/dc_i) sum_(j<i) gamma[k][i][j] F[j] for the n x ld planes, with
   F device [s-1][n][ld] and rho device [n_gamma][n][ld]; 1 <= stage < s. */
mri_status mri_forcing_assemble(const mri_table *t, int stage, int n, int ld, const double *F,
                                double *rho, mri_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* MRI_SURROGATE_H */
