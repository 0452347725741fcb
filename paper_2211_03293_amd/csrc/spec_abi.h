// spec_abi.h -- argument structures shared by the host launcher (libmri) and
// the run-time compiled kernels of spec_kernels.inc.  Plain C layout only.
#pragma once

struct ZvOpts {
    double rtol, atol_Y, atol_T;
    int max_steps;
};

struct BatchArgs {
    const double *yin;
    double *yout;
    const double *rho;
    const long long *set_off;           // [n_sets + 1]
    const double *set_L;                // [n_sets]
    int *status;
    int *steps;                         // accepted steps per cell (nullable)
    int *rejects;                       // rejected steps per cell (nullable)
    unsigned long long *counter;        // next unclaimed cell
    unsigned long long *lane_steps;     // useful lane-steps (nullable)
    unsigned long long *issued_steps;   // issued lane-steps (nullable)
    long long n_total;
    long long ld;
    int n_sets;
    ZvOpts o;
};
