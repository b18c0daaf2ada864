// Device-side gather of the matrices the no-click conditioning starts from
// (csrc/tor_gather.hip).
#pragma once
#include <hip/hip_runtime.h>

// One query: sigma_Q over the rows g[0..R) of a state's covariance (global
// quadrature indices, clicked modes first, then the no-click modes), packed
// lower, double-double words (the diagonal's + 1/2 formed exactly), with the
// row [0, mean[g]] first when mean is not null.  Written to out[0 ..
// EN(R/2, mean != null)); the job's entries are the launch's flat entries
// begin .. begin + count.
struct GatherJob {
    const double *cov;   // 2m x 2m, row-major (device)
    const double *mean;  // 2m (device), or null for a zero-mean state
    const int *g;        // R row indices (device)
    void *out;           // packed output (device)
    long long begin;     // first flat entry of this job
    int m;
    int R;
};

// jobs sorted by begin; total = sum of the jobs' entry counts.
hipError_t tor_launch_cond_gather(const GatherJob *jobs, int njobs, long long total, hipStream_t st);

// Screen of a caller's covariance over the rows and columns g[0..R) (global
// quadrature indices): out[0] receives the bits of max |cov[a][b]|, out[1] is
// set to 1 if an entry is not finite, out[2] receives the bits of
// max |cov[a][b] - cov[b][a]| (a, b over g); out must hold zeros before.  The
// caller compares out[2] with 1e-12 out[0], the host's symmetry test.
hipError_t tor_launch_cov_screen(const double *cov, int m, const int *g, int R, unsigned long long *out,
                                 hipStream_t st);
