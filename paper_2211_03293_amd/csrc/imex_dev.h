// imex_dev.h -- launchers of the IMEX-MRI-GARK kernels (imex_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

// Slow evaluations per partition (stages j < i) and forcing terms a
// combination can take.
constexpr int IMEX_JMAX = 12;
constexpr int IMEX_KMAX = 4;

// Coefficients of one combination: out[k] = base + sum_j (e[k][j] FE_j + i[k][j] FI_j).
struct ImexCoef {
    double e[IMEX_KMAX][IMEX_JMAX];
    double i[IMEX_KMAX][IMEX_JMAX];
};

// Per-component conjugate-gradient scalars.
struct CgScalars {
    double rr, bb, alpha, beta;
};

// n x ld planes (FE, FI: nj planes each, plane stride n * ld); cells below
// n_cells of every component; base nullable; out: n_out planes.
hipError_t launch_imex_combine(int n, int n_cells, int ld, int n_out, int nj, const double *FE,
                               const double *FI, const ImexCoef &coef, const double *base,
                               double *out, hipStream_t s);

// Blocks per component of the stencil and vector kernels (partial-sum counts).
int cg_apply_blocks(int nx, int ny, int nz);
int cg_vec_blocks(int n_cells);

hipError_t launch_cg_apply(int nx, int ny, int nz, int n_comp, int ld, double aD, double dx,
                           const double *p, double *q, const int *done, double *part,
                           hipStream_t s);
hipError_t launch_cg_init(int n_comp, int n_cells, int ld, const double *b, const double *q,
                          double *r, double *p, double *part_rr, double *part_bb, hipStream_t s);
hipError_t launch_cg_update(int n_comp, int n_cells, int ld, const CgScalars *sc, const int *done,
                            double *x, double *r, const double *p, const double *q, double *part,
                            hipStream_t s);
hipError_t launch_cg_dir(int n_comp, int n_cells, int ld, const CgScalars *sc, const int *done,
                         const double *r, double *p, hipStream_t s);
hipError_t launch_cg_reduce(int mode, int n_comp, int nb, const double *part, const double *part2,
                            double tol2, CgScalars *sc, int *done, hipStream_t s);
hipError_t launch_copy_planes(int n_comp, int n_cells, int ld, const double *src, double *dst,
                              hipStream_t s);
hipError_t launch_fill_i32(int *p, int n, int v, hipStream_t s);
