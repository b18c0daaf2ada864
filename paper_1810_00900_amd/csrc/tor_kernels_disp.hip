// Wave-tier kernels of displaced states: the same subset tree as the zero-mean
// kernels, over packed matrices that carry the mean vector as their first row
// (each pivot's factor gains the overlap term of its conditioned mean; see
// make_pivot_m).  A translation unit of its own so that it compiles in
// parallel with the zero-mean instantiations.
#include "tor_wave.hpp"

#pragma clang fp contract(off)

hipError_t tor_launch_wave_disp(int is_dd, int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                                int grid_cap, hipStream_t st, const LaunchDims *dyn) {
    return is_dd ? tor::launch_wave_S<dd, 1>(J, jobs, njobs, total, pool, grid_cap, st, dyn)
                 : tor::launch_wave_S<double, 1>(J, jobs, njobs, total, pool, grid_cap, st, dyn);
}
