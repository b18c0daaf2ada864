// Wave-tier kernels of the information form: full patterns of an inverted
// displaced state are subset sums of G = sigma_Q^-1 over the clicked modes
// with the row h = (sigma_Q^-1 mu) over them first, each pivot's factor
// carrying exp(+|w|^2 / 2) instead of the overlap exp(-|w|^2 / 2) (see
// make_pivot_m).  A translation unit of its own so that it compiles in
// parallel with the other instantiations.
#include "tor_wave.hpp"

#pragma clang fp contract(off)

hipError_t tor_launch_wave_info(int is_dd, int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                                int grid_cap, hipStream_t st, const LaunchDims *dyn) {
    return is_dd ? tor::launch_wave_S<dd, -1>(J, jobs, njobs, total, pool, grid_cap, st, dyn)
                 : tor::launch_wave_S<double, -1>(J, jobs, njobs, total, pool, grid_cap, st, dyn);
}
