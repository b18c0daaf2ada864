// Gather of sigma_Q over a query's observed modes on the device, from the
// state's device copy of the covariance: what the host would otherwise pack
// and copy for every query with no-click modes (the start of the vacuum
// conditioning of Eq. MatrixUpdate).  The words are formed exactly as the
// host forms them (the diagonal's sigma + 1/2 by an error-free sum, the mean
// row as binary64 words), so the conditioned matrices, and every result, are
// bitwise those of the host-packed path.
#include <hip/hip_runtime.h>

#include "dd.hpp"
#include "tor_gather.h"
#include "tor_tree.hpp"

#pragma clang fp contract(off)

namespace tor {

__global__ __launch_bounds__(256) void cond_gather_kernel(const GatherJob *__restrict__ jobs, int njobs,
                                                          long long total) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        int lo = 0, hi = njobs - 1;  // last job with begin <= t
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (jobs[mid].begin <= t) lo = mid;
            else hi = mid - 1;
        }
        const GatherJob &J = jobs[lo];
        const int e = (int)(t - J.begin);
        int a, b;
        unpack(e, a, b);
        const int o = J.mean ? 1 : 0;
        dd x;
        if (o && b == 0) {  // the mean column (0 at the corner)
            x = dd_from(a == 0 ? 0.0 : J.mean[J.g[a - 1]]);
        } else {
            const int ga = J.g[a - o], gb = J.g[b - o];
            const int r = ga > gb ? ga : gb, c = ga > gb ? gb : ga;
            const double v = J.cov[(size_t)r * (size_t)(2 * J.m) + (size_t)c];
            if (ga == gb) two_sum(v, 0.5, x.hi, x.lo);
            else x = dd_from(v);
        }
        ((dd *)J.out)[e] = x;
    }
}

}  // namespace tor

hipError_t tor_launch_cond_gather(const GatherJob *jobs, int njobs, long long total, hipStream_t st) {
    if (njobs < 1 || total < 1) return hipSuccess;
    const long long blocks = (total + 255) / 256;
    const unsigned g = (unsigned)(blocks < 262144 ? blocks : 262144);
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::cond_gather_kernel, dim3(g), dim3(256), 0, st, jobs, njobs, total);
    return hipGetLastError();
}
