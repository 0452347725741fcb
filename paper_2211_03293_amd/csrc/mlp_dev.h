// mlp_dev.h -- surrogate MLP: fixed architecture and kernel launchers.
//
// Inputs (MLP_FEAT = 89, padded to MLP_KPAD = 96): log max(Y_k, 1e-30) for the
// MLP_NS = 21 species, T, the MLP_NPOLY = 3 forcing-polynomial coefficients of
// each of the MLP_NC = 22 components (zero where the table has fewer terms),
// and log L (the stage length).  Three hidden layers of MLP_HID = 256 with SiLU,
// output MLP_NC = 22 standardized stage increments (padded to 32 rows): for a
// species the log-increment log(Y1 + eps) - log(Y0 + eps) with eps = MLP_EPS
// (Y0 clamped at 0), so that an output error is a relative error of Y + eps;
// for T the plain increment T1 - T0.
// Statistics buffer `stats` (FP64): [x_mean (89), x_inv_std (89), y_mean (22),
// y_inv_std (22), y_std (22)].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MLP_NS 21
#define MLP_NC 22
#define MLP_NPOLY 3
#define MLP_FEAT (MLP_NS + 1 + MLP_NPOLY * MLP_NC + 1)
#define MLP_KPAD 96
#define MLP_K0_IN 128   // first-layer row length in the inference weight stream
#define MLP_HID 256
#define MLP_OUT_PAD 32
#define MLP_STATS (2 * MLP_FEAT + 3 * MLP_NC)
#define MLP_EPS 1e-8

// C = op(A) op(B); with a partial buffer (part_elems floats) long-K products
// with few output tiles are split over K and reduced deterministically.
hipError_t mlp_gemm(int M, int N, int K, const uint16_t *A, int lda, int transA,
                    const uint16_t *B, int ldb, int transB, float *C, int ldc, hipStream_t s,
                    float *part = nullptr, size_t part_elems = 0);
hipError_t mlp_bias_act(int rows, int N, float *Z, const float *bias, int act, uint16_t *Aout,
                        hipStream_t s);
hipError_t mlp_mse_grad(int rows, int N, const float *Y, const float *T, float *dZ, uint16_t *dZq,
                        double *loss, hipStream_t s);
hipError_t mlp_silu_bwd(long long n, const float *dA, const float *Z, float *dZ, uint16_t *dZq,
                        hipStream_t s);
hipError_t mlp_colsum(int rows, int N, const float *dZ, float *db, hipStream_t s,
                      float *part = nullptr, size_t part_elems = 0);
hipError_t mlp_adam(long long n, float *w, const float *g, float *m, float *v, uint16_t *wq,
                    float lr, float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t mlp_to_bf16(long long n, const float *x, uint16_t *y, hipStream_t s);
hipError_t mlp_featurize(int B, const int *idx, long long ld, const double *Y0, int n_poly,
                         const double *RHO, const double *Lv, const double *Yb,
                         const double *Y1, const double *stats, uint16_t *X, float *T,
                         hipStream_t s);
hipError_t mlp_stats(long long N, long long ld, const double *Y0, int n_poly, const double *RHO,
                     const double *Lv, const double *Yb, const double *Y1, double *part,
                     int n_blocks, double *stats, hipStream_t s);
hipError_t mlp_infer(const double *yin, const double *base, double *yout, const double *rho,
                     const uint16_t *const *W, const float *const *b, const double *stats,
                     long long ld, int n_cells, int n_poly, double L, hipStream_t s);
// mlp_infer followed by mlp_gate's check in one launch (base = vc; the network
// states are not written, accepted cells go to yout as with mlp_gate)
hipError_t mlp_infer_gate(const double *yin, const double *vc, const double *vh,
                          const double *rho, const uint16_t *const *W, const float *const *b,
                          const double *stats, long long ld, int n_cells, int n_poly, double L,
                          const int *status_c, double rich, double tol, double *yout,
                          int *used_fallback, double *gval, int *status, int *list,
                          unsigned int *count, hipStream_t s);
hipError_t mlp_gate(int n_cells, long long ld, const double *yin, const double *rho, int n_poly,
                    double L, const double *vc, const double *vh, const double *vn,
                    const int *status_c, double rich, double tol, double *yout, int *used_fallback,
                    double *gval, int *status, int *list, unsigned int *count, hipStream_t s);
hipError_t mlp_gather(int n_planes, const unsigned int *count, const int *list, long long n_max,
                      const double *src, long long lds, double *dst, long long ldd, hipStream_t s);
hipError_t mlp_scatter(int n_planes, const unsigned int *count, const int *list, long long n_max,
                       const double *src, long long lds, double *dst, long long ldd, hipStream_t s);
// *p = 0 by a one-thread kernel (no memset node when the stream is captured).
hipError_t mlp_zero_u32(unsigned int *p, hipStream_t s);
hipError_t mlp_scatter_i32(const unsigned int *count, const int *list, long long n_max,
                           const int *src, int *dst, hipStream_t s);
