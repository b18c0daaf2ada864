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

// Every workgroup reduces its share in LDS and adds it with one atomic per
// word (non-negative doubles order as their bit patterns).
__global__ __launch_bounds__(256) void cov_screen_kernel(const double *__restrict__ cov, int m,
                                                         const int *__restrict__ g, int R,
                                                         unsigned long long *__restrict__ out) {
    __shared__ double sa[256], ss[256];
    __shared__ int sn[256];
    const long long total = (long long)R * R, ld = 2LL * m;
    double amax = 0.0, asym = 0.0;
    int bad = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < total;
         i += (long long)gridDim.x * blockDim.x) {
        const int a = (int)(i / R), b = (int)(i - (long long)a * R);
        const double v = cov[(long long)g[a] * ld + g[b]];
        bad |= !isfinite(v);
        amax = fmax(amax, fabs(v));
        if (b < a) asym = fmax(asym, fabs(v - cov[(long long)g[b] * ld + g[a]]));
    }
    sa[threadIdx.x] = amax;
    ss[threadIdx.x] = asym;
    sn[threadIdx.x] = bad;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            sa[threadIdx.x] = fmax(sa[threadIdx.x], sa[threadIdx.x + h]);
            ss[threadIdx.x] = fmax(ss[threadIdx.x], ss[threadIdx.x + h]);
            sn[threadIdx.x] |= sn[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(sa[0]));
        if (sn[0]) atomicOr(&out[1], 1ULL);
        atomicMax(&out[2], (unsigned long long)__double_as_longlong(ss[0]));
    }
}

}  // namespace tor

hipError_t tor_launch_cov_screen(const double *cov, int m, const int *g, int R, unsigned long long *out,
                                 hipStream_t st) {
    const long long total = (long long)R * R;
    if (total < 1) return hipSuccess;
    const long long blocks = (total + 255) / 256;
    const unsigned gr = (unsigned)(blocks < 4096 ? blocks : 4096);
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::cov_screen_kernel, dim3(gr), dim3(256), 0, st, cov, m, g, R, out);
    return hipGetLastError();
}

hipError_t tor_launch_cond_gather(const GatherJob *jobs, int njobs, long long total, hipStream_t st) {
    if (njobs < 1 || total < 1) return hipSuccess;
    const long long blocks = (total + 255) / 256;
    const unsigned g = (unsigned)(blocks < 262144 ? blocks : 262144);
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::cond_gather_kernel, dim3(g), dim3(256), 0, st, jobs, njobs, total);
    return hipGetLastError();
}
