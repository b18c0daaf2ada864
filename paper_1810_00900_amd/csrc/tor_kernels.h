// Internal launch interface between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TOR_MAX_N 32

// A node of the subset tree: its packed matrix starts at pool + off (in
// scalars; the node uses the leading r-mode prefix), and the signed product of
// the pivot factors q along its path, coef = prod (-q) as a double-double, and
// acoef = prod q (binary64) for the magnitude sum.
struct NodeDesc {
    unsigned long long off;
    double coef_hi, coef_lo;
    double acoef;
};

// Partial sums of one task: T (double-double) and A (binary64).
struct Partial {
    double t_hi, t_lo, a, pad;
};

#ifdef __cplusplus
extern "C" {
#endif
hipError_t tor_launch_wave(int is_dd, int J, const NodeDesc *tasks, long long ntasks, const void *pool,
                           Partial *out, int grid_cap, hipStream_t st);
hipError_t tor_launch_expand(int is_dd, const NodeDesc *par, long long npar, int r, void *pool,
                             unsigned long long child_base, NodeDesc *chi, int grid_cap, hipStream_t st);
hipError_t tor_launch_reduce(const Partial *in, long long n, long long chunk, Partial *out, hipStream_t st);
int tor_wave_lds_bytes(int is_dd, int J);
#ifdef __cplusplus
}
#endif
