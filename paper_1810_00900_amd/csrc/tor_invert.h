// Launchers of the per-state inverse of sigma_Q (csrc/tor_invert.hip).
#pragma once
#include <hip/hip_runtime.h>

// Largest state the inverse is formed for (2m x 2m packed on the device and
// kept on the host: 537 MB in quad-double at this size).
#define TOR_INVERT_MAX_MODES 2048

// One symmetric sweep of the packed lower 2m x 2m matrix A (row-major lower,
// entry (a, b), a >= b, at a(a+1)/2 + b) on the 2x2 block of mode k: the
// columns launch writes the scaled pivot columns to cols (2 * 2m words) and the
// pivot's scalars to piv (3 words), and multiplies acc[0] + acc[1] (a
// double-word) by det(block)^-1/2 and adds log det(block)^-1/2 to acc[2]; the
// update launch then rewrites every entry of A.  After the sweeps of all m
// modes in any order A holds -A0^-1.  is_qd: the words are quad-double,
// else double-double.
hipError_t tor_launch_sweep(int is_qd, void *A, int m, int k, void *cols, void *piv, double *acc, hipStream_t st);
// A <- packed sigma_Q (double-double or quad-double words) from the row-major
// 2m x 2m covariance cov (device); acc <- (1, 0, 0)
hipError_t tor_launch_pack_sigq(int is_qd, const double *cov, int m, void *A, double *acc, hipStream_t st);
// A <- -A over the E(m) packed words
hipError_t tor_launch_negate(int is_qd, void *A, int m, hipStream_t st);
