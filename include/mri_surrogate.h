/*
 * mri_surrogate.h -- learned fast-stage surrogate of libmri: a small MLP that
 * predicts the stage increment of the modified fast IVP (the stage solve of
 * the MRI algorithm, Sec. 2.1 step 2b), trained on stages of the plain FP64
 * method, run with BF16 MFMA kernels (FP32 accumulation), and backed by the
 * plain FP64 fast-stage solve wherever a step-doubling check of its prediction
 * exceeds a tolerance.  The paper has no surrogate; it is an addition to the
 * method, and the plain solve stays the reference for every result.
 *
 * Architecture (fixed for inference): 89 inputs -- log max(Y_k, 1e-30) for 21
 * species, T, the 3 forcing-polynomial coefficients of each of the 22 state
 * components (zero where the coupling table has fewer terms), log L (stage
 * length) -- standardized with training-set statistics; 3 hidden layers of
 * 256 with SiLU; 22 outputs = standardized stage increments: for a species
 * log(Y(L) + 1e-8) - log(Y(0) + 1e-8) (Y(0) clamped at 0), so that an output
 * error is a relative error of Y + 1e-8 (the floor of the gate below); for T
 * the plain increment T(L) - T(0).
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
#define MRI_MLP_OUTPUTS 22       /* stage increments of the 22 components  */
#define MRI_MLP_STATS (2 * 89 + 3 * 22)
/* stats layout (FP64): x_mean[89], x_inv_std[89], y_mean[22], y_inv_std[22],
   y_std[22] (inverse std 1 where a feature is constant); y_* describe the
   increments defined above. */

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
/* Y0[c*ld + s] and Y1[c*ld + s] (c < 22) the stage start and end states,     */
/* RHO[(p*22 + c)*ld + s] (p < n_poly) the forcing coefficients, Lv[s] the    */
/* stage length.                                                              */
/* ------------------------------------------------------------------------- */
/* Feature / increment statistics over n samples into stats (device FP64
   [MRI_MLP_STATS]).  Deterministic (fixed reduction order). */
mri_status mri_mlp_feature_stats(int64_t n, int64_t ld, const double *Y0, int n_poly,
                                 const double *RHO, const double *Lv, const double *Y1,
                                 double *stats, mri_stream_t stream);
/* Standardized features X (device bf16 [batch][96]) and targets T (nullable,
   device f32 [batch][22]) of the samples idx[0..batch) (idx NULL: 0..batch). */
mri_status mri_mlp_featurize(int batch, const int32_t *idx, int64_t ld, const double *Y0,
                             int n_poly, const double *RHO, const double *Lv, const double *Y1,
                             const double *stats, uint16_t *X, float *T, mri_stream_t stream);

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

/* One fused inference: y_out = y_in advanced by the predicted increment over a stage of
   length L with forcing rho (device [n_poly][22][ld], n_poly <= 3).
   half = 0 the full stage; 1 / 2 the first / second half (length L/2, forcing
   re-expanded on the half).  y_out must not alias y_in. */
mri_status mri_surrogate_infer(const mri_surrogate *s, int n_cells, int ld, const double *y_in,
                               double *y_out, int n_poly, const double *rho, double L, int half,
                               mri_stream_t stream);

mri_status mri_surrogate_workspace_bytes(int n_cells, int ld, int n_poly, size_t *bytes);

/* Gated surrogate stage: predicts the stage end once over L and twice over
   L/2 (step doubling); a cell is accepted when max(D, I) <= gate_tol with
   D = max_c |full_c - doubled_c| / max(|doubled_c|, floor_c) (floor 1e-8 for
   mass fractions, 0 for T) and I the residual of the mass-sum invariant
   |sum_k (doubled_k - y_in_k) - L sum_p sum_k rho_(p,k) / (p + 1)| /
   sum_k |y_in_k| (the chemistry conserves sum_k Y_k, so the sum changes only
   by the integral of the forcing); an accepted cell takes the doubled
   prediction;
   every other cell is compacted and integrated by the plain FP64 fast stage
   (mech, fallback options) and scattered back.  used_fallback (nullable,
   device int32 [n_cells]) marks fallback cells; gate_value (nullable, device
   float [n_cells]) receives the check value; n_fallback (nullable, host)
   receives their number (the call synchronizes the stream once to size the
   fallback launch).  y_out may alias y_in. */
mri_status mri_surrogate_stage(const mri_surrogate *s, const mri_mech *mech,
                               const mri_fast_opts *fallback, double gate_tol, int n_cells, int ld,
                               const double *y_in, double *y_out, int n_poly, const double *rho,
                               double L, int32_t *used_fallback, float *gate_value,
                               int64_t *n_fallback, void *ws, size_t ws_bytes,
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
