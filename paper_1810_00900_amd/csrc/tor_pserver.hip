// Persistent request loop: one long-running kernel whose workgroups take the
// work units of probability queries and of chain-rule sampling batches as the
// host publishes them, so that requests arriving while others run are admitted
// into the device's work at once (continuous batching on the device).
//
// A probability query (Sec. II of arXiv:1810.00900: the signed sum over the
// subsets of the clicked modes of the vacuum probabilities of Eq. (prob)) is
// the subset tree over Sigma_C, split exactly as the batched path splits it:
// the top n - J decisions are taken by Schur-complement updates (Eq.
// MatrixUpdate) and the J-mode nodes below are the wave-tier tasks.  A unit of
// the query is the subtree below one node of depth g: its workgroup gathers
// Sigma_C from the state's device copy, applies the unit's g decisions, walks
// the next t decisions depth first (one buffer per level in global memory) and
// evaluates every task with the wave tier, writing each task's partial sum.
// The arithmetic of every node and task is that of the batched path, and the
// last unit of the query sums the task partials in the batched path's
// reduction order, so a result equals tor_batch's bitwise, whatever the other
// requests in flight.  A sampling unit is one chain (tor_chain.hpp).
//
// Waiting: a workgroup waits only for new work, polling a device copy of the
// host's control block (one workgroup at a time refreshes the copy).  The
// kernel exits on the host's stop flag, or as a whole once every running
// workgroup has been idle_ticks without work (one of them closes the launch;
// the others leave when they see it, each after the unit it holds); the host
// launches the kernel again when work arrives, queued behind a launch that is
// closing.  Units never wait for each other.
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "dd.hpp"
#include "tor_chain.hpp"
#include "tor_kernels.h"
#include "tor_tree.hpp"
#include "tor_wave.hpp"

#pragma clang fp contract(off)

namespace tor {

// Chain working set inside the shared LDS region: the chain kernel's layout
// (its wave-tier part first, whose packed-index table is the same as the
// probability tasks').
struct PsChainLds {
    unsigned char raw[ChainLds<double, 0>::wave_bytes];
    double gbuf[3][EN(TOR_CHAIN_MAX, 0)];
    double vt[4 * TOR_CHAIN_MAX];
    int Cl[TOR_CHAIN_MAX + 1];
};

// Reduction working set (256 sums, as reduce_kernel's 256 threads), placed
// after the packed-index table.
struct PsReduceLds {
    unsigned char skip[512];
    dd sT[256];
    double sA[256];
};

// Byte offset of the prefix buffer in the shared LDS region: after the
// packed-index table, room for 32 modes (E(32) double-doubles).
constexpr int kPsPrefixOffset = 512;

union PsLds {
    TopSmem<dd, 0, 2> top;  // largest probability task (11 modes); smaller tasks use its prefix
    PsChainLds chain;
    PsReduceLds red;
    unsigned char prefix[kPsPrefixOffset + EN(TOR_MAX_N, 0) * sizeof(dd)];  // the walk's prefix matrix
};

using PsWaveDD = WaveSmem<dd, 9, 0>;
using PsWaveF64 = WaveSmem<double, 9, 0>;
static_assert(offsetof(PsWaveDD, mat) == offsetof(PsWaveF64, mat),
              "the probability and chain working sets share the packed-index table");

// Ordering of a wave's global-memory stores before its own later loads of
// them (the per-workgroup scratch): workgroup-scope release and acquire.
__device__ __forceinline__ void ps_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Include child of the r-mode node `in` (global memory) into `out`: the
// expansion's Schur update, operation for operation.
__device__ __forceinline__ Pivot<dd> ps_schur(const dd *in, int r, dd *out, dd *vt, int lane) {
    const int R = 2 * r, RC = R - 2, EC = EN(r - 1, 0);
    const Pivot<dd> pv = make_pivot_m<dd, 0>(in, R - 2, R - 1);
    for (int c = lane; c < RC; c += 64) {
        const dd c0 = in[pidx(R - 2, c)];
        vt[c] = mul_s(c0, pv.s1);
        vt[RC + c] = mul_s(sub_mul(in[pidx(R - 1, c)], pv.l, c0), pv.s2);
    }
    wave_sync();
    for (int e = lane; e < EC; e += 64) {
        int a, b;
        unpack(e, a, b);
        out[e] = sub_dot2(in[e], vt[a], vt[b], vt[RC + a], vt[RC + b]);
    }
    ps_sync();
    return pv;
}

// Sigma_C of the request (packed lower, exact double-double) into out: sigma_Q
// over the clicked modes from the covariance (sigma + I/2, the diagonal by an
// exact two-sum), or G = sigma_Q^-1 over them from the inverse.
__device__ __forceinline__ void ps_gather(const PsReq &R, dd *out, int lane) {  // out: LDS
    const int E = EN(R.n, 0);
    const long long ld = 2LL * R.m;
    for (int e = lane; e < E; e += 64) {
        int a, b;
        unpack(e, a, b);
        const long long ga = 2LL * R.C[a >> 1] + (a & 1), gb = 2LL * R.C[b >> 1] + (b & 1);  // ga >= gb
        if (R.jac) {
            out[e] = R.inv[ga * (ga + 1) / 2 + gb];
        } else {
            const double v = R.cov[ga * ld + gb];
            dd o;
            if (ga == gb) two_sum(v, 0.5, o.hi, o.lo);
            else o = dd_from(v);
            out[e] = o;
        }
    }
    wave_sync();
}

// Include child of the r-mode node m (LDS) in place (the expansion's update).
__device__ __forceinline__ Pivot<dd> ps_schur_lds(dd *m, int r, dd *vt, int lane) {
    const int R = 2 * r, RC = R - 2, EC = EN(r - 1, 0);
    const Pivot<dd> pv = make_pivot_m<dd, 0>(m, R - 2, R - 1);
    for (int c = lane; c < RC; c += 64) {
        const dd c0 = m[pidx(R - 2, c)];
        vt[c] = mul_s(c0, pv.s1);
        vt[RC + c] = mul_s(sub_mul(m[pidx(R - 1, c)], pv.l, c0), pv.s2);
    }
    wave_sync();
    for (int e = lane; e < EC; e += 64) {
        int a, b;
        unpack(e, a, b);
        m[e] = sub_dot2(m[e], vt[a], vt[b], vt[RC + a], vt[RC + b]);
    }
    wave_sync();
    return pv;
}

// One wave-tier task of J <= TOR_PS_TASK_MAX modes at node (global memory).
__device__ __forceinline__ void ps_task(PsLds &L, int J, const dd *node, dd c, double a, int lane, dd &T,
                                        double &A) {
    switch (J) {
    case 1: wave_task<dd, 1, 0>(*reinterpret_cast<WaveSmem<dd, 1, 0> *>(&L), node, c, a, lane, T, A); break;
    case 2: wave_task<dd, 2, 0>(*reinterpret_cast<WaveSmem<dd, 2, 0> *>(&L), node, c, a, lane, T, A); break;
    case 3: wave_task<dd, 3, 0>(*reinterpret_cast<WaveSmem<dd, 3, 0> *>(&L), node, c, a, lane, T, A); break;
    case 4: wave_task<dd, 4, 0>(*reinterpret_cast<WaveSmem<dd, 4, 0> *>(&L), node, c, a, lane, T, A); break;
    case 5: wave_task<dd, 5, 0>(*reinterpret_cast<WaveSmem<dd, 5, 0> *>(&L), node, c, a, lane, T, A); break;
    case 6: wave_task<dd, 6, 0>(*reinterpret_cast<WaveSmem<dd, 6, 0> *>(&L), node, c, a, lane, T, A); break;
    case 7: wave_task<dd, 7, 0>(*reinterpret_cast<WaveSmem<dd, 7, 0> *>(&L), node, c, a, lane, T, A); break;
    case 8: wave_task<dd, 8, 0>(*reinterpret_cast<WaveSmem<dd, 8, 0> *>(&L), node, c, a, lane, T, A); break;
    case 9: wave_task<dd, 9, 0>(L.top.w, node, c, a, lane, T, A); break;
    case 10:
        wave_task_top<dd, 10, 0>(*reinterpret_cast<TopSmem<dd, 0, 1> *>(&L), node, c, a, lane, T, A);
        break;
    default: wave_task_top<dd, 11, 0>(L.top, node, c, a, lane, T, A); break;
    }
}

struct PsPath {  // node of each level of the depth-first walk (wave-uniform)
    const dd *node[TOR_PS_LMAX + 1];
    dd c[TOR_PS_LMAX + 1];
    double a[TOR_PS_LMAX + 1];
};

// LDS of the kernel: four workgroups per CU (160 KiB).
static_assert(kPsPrefixOffset + EN(TOR_MAX_N, 0) * (int)sizeof(dd) <= (int)sizeof(PsLds),
              "the prefix buffer fits the shared LDS region");
static_assert(sizeof(PsLds) + sizeof(PsReq) + sizeof(PsPath) + 2 * (2 * TOR_MAX_N - 2) * sizeof(dd) + 64 <=
                  40 * 1024,
              "four workgroups per CU");

// Unit u of a probability request: the subtree below the depth-g node whose
// decisions are u's bits (most significant first; 1 = include), its tasks
// (u << t) .. (u << t) + 2^t - 1 in the batched path's order.
__device__ __attribute__((noinline)) void ps_prob_unit(const PsReq &R, long long u, dd *ws, PsLds &L, dd *vt,
                                                      PsPath &path, int lane) {
    constexpr long long EW = TOR_MAX_N * (2 * TOR_MAX_N + 1);
    // the unit's g decisions in LDS (the task working set is free until the
    // first task; the packed-index table before it is kept): Sigma_C gathered
    // there, each include decision an in-place Schur update (an entry of the
    // child needs only itself and the pivot columns, set aside in vt), the
    // arithmetic of the expansion's update
    dd *lm = reinterpret_cast<dd *>(reinterpret_cast<unsigned char *>(&L) + kPsPrefixOffset);
    ps_gather(R, lm, lane);
    dd c = dd_from(1.0);
    double a = 1.0;
    int r = R.n;
    for (int k = 0; k < R.g; ++k, --r) {
        if ((u >> (R.g - 1 - k)) & 1) {
            const Pivot<dd> pv = ps_schur_lds(lm, r, vt, lane);
            c = dd_neg(coef_mul(c, pv.q));
            a = a * hi_of(pv.q);
        }
    }
    // the unit's node to global memory: the root of its depth-first walk
    dd *root = ws;
    for (int e = lane; e < EN(r, 0); e += 64) root[e] = lm[e];
    ps_sync();
    const int t = R.t;
    if (lane == 0) {
        path.node[0] = root;
        path.c[0] = c;
        path.a[0] = a;
    }
    wave_sync();
    for (long long q = 0; q < (1LL << t); ++q) {
        // levels from the first decision where q differs from q - 1
        const int f = q == 0 ? 0 : t - 1 - __builtin_ctzll((unsigned long long)q);
        for (int k = f; k < t; ++k) {
            const dd *par = path.node[k];
            const dd pc = path.c[k];
            const double pa = path.a[k];
            wave_sync();
            if ((q >> (t - 1 - k)) & 1) {
                dd *out = ws + (1 + k) * EW;
                const Pivot<dd> pv = ps_schur(par, r - k, out, vt, lane);
                if (lane == 0) {
                    path.node[k + 1] = out;
                    path.c[k + 1] = dd_neg(coef_mul(pc, pv.q));
                    path.a[k + 1] = pa * hi_of(pv.q);
                }
            } else if (lane == 0) {
                path.node[k + 1] = par;
                path.c[k + 1] = pc;
                path.a[k + 1] = pa;
            }
            wave_sync();
        }
        dd T;
        double A;
        ps_task(L, R.J, path.node[t], path.c[t], path.a[t], lane, T, A);
        if (lane == 0) {
            Partial p;
            p.t_hi = T.hi;
            p.t_lo = T.lo;
            p.a = A;
            p.pad = 0.0;
            R.part[(u << t) + q] = p;
        }
        wave_sync();
    }
}

// A sampling unit: one chain.  The two kinds of unit are kept out of line so
// that their register allocations stay apart (each as in its own kernel).
__device__ __attribute__((noinline)) void ps_chain_unit(const ChainParams &P, int ci, PsChainLds &L, int lane) {
    run_chain<double, TOR_CHAIN_MAX, 0>(P, ci, L.raw, L.gbuf[0], L.gbuf[1], L.vt, L.Cl, lane);  // gbuf[1], gbuf[2]
}

// Sum of the request's task partials in the batched path's order: stages of
// TOR_REDUCE_CHUNK partials per block, each block summed by 256 strided
// sequential sums (four per lane here) and a fixed pairwise tree.
__device__ __forceinline__ Partial ps_reduce(const PsReq &R, PsLds &L, int lane) {
    const Partial *in = R.part;
    Partial *out = R.part + R.tasks;
    long long count = R.tasks;
    dd *sT = L.red.sT;
    double *sA = L.red.sA;
    while (count > 1) {
        const long long nb = (count + TOR_REDUCE_CHUNK - 1) / TOR_REDUCE_CHUNK;
        for (long long b = 0; b < nb; ++b) {
            const long long lo = b * TOR_REDUCE_CHUNK;
            const long long hi = lo + TOR_REDUCE_CHUNK < count ? lo + TOR_REDUCE_CHUNK : count;
            for (int v = lane; v < 256; v += 64) {
                dd T = dd_from(0.0);
                double A = 0.0;
                for (long long k = lo + v; k < hi; k += 256) {
                    const Partial p = in[k];
                    T = dd_add(T, dd_make(p.t_hi, p.t_lo));
                    A += p.a;
                }
                sT[v] = T;
                sA[v] = A;
            }
            wave_sync();
            for (int s = 128; s > 0; s >>= 1) {
                for (int v = lane; v < s; v += 64) {
                    sT[v] = dd_add(sT[v], sT[v + s]);
                    sA[v] = sA[v] + sA[v + s];
                }
                wave_sync();
            }
            if (lane == 0) {
                Partial p;
                p.t_hi = sT[0].hi;
                p.t_lo = sT[0].lo;
                p.a = sA[0];
                p.pad = 0.0;
                out[b] = p;
            }
            wave_sync();
        }
        ps_sync();
        in = out;
        out += nb;
        count = nb;
    }
    return in[0];
}

constexpr int kPsMaxBackoff = 3;  // log2 of the most sleeps between idle polls

// Move the claim cursor past request k (lane 0; a failed exchange means
// another workgroup moved it).
__device__ __forceinline__ void ps_advance(const PsParams &P, unsigned long long k) {
    unsigned long long kk = k;
    __hip_atomic_compare_exchange_strong(&P.dev->cur, &kk, k + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
}

// Publish a finished request: the result words, the claim cursor moved past
// it, the slot's completion count made ready for request seq + TOR_PS_SLOTS
// (its claim counter is reset once that request is published), then the
// completion word (system-scope release, read by the host).  Lane 0 only.
__device__ __forceinline__ void ps_publish(const PsParams &P, const PsReq &R, const Partial *res) {
    const int slot = (int)(R.seq % TOR_PS_SLOTS);
    if (res) {
        P.res[slot].t_hi = res->t_hi;
        P.res[slot].t_lo = res->t_lo;
        P.res[slot].a = res->a;
    }
    ps_advance(P, (unsigned long long)R.seq);
    __hip_atomic_store(&P.dev->done[slot], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&P.res[slot].done, (unsigned long long)R.seq + 1ULL, __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ __forceinline__ void ps_mirror(const PsParams &P);

// Copy the host's control block into the per-XCD copies if this workgroup
// refreshes (one of the eight designated ones, or at its longest backoff) and
// the refresh period has passed (lane 0).  Returns whether requests beyond k
// were found; sets stop when the host has asked the kernel to stop.
__device__ __forceinline__ bool ps_refresh(const PsParams &P, unsigned long long k, int backoff, bool &stop) {
    if (!(blockIdx.x < 8 || backoff == kPsMaxBackoff)) return false;
    const unsigned long long now = wall_clock64();
    unsigned long long last = __hip_atomic_load(&P.dev->refresh, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (now - last <= (unsigned long long)P.refresh_ticks ||
        !__hip_atomic_compare_exchange_strong(&P.dev->refresh, &last, now, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT))
        return false;
    const unsigned long long hp = __hip_atomic_load(&P.host->published, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
    const unsigned int hs = __hip_atomic_load(&P.host->stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
    const unsigned long long v = hp | (hs ? 1ULL << 63 : 0ULL);
    for (int x = 0; x < 8; ++x)
        __hip_atomic_fetch_max(&P.dev->pubx[x][0], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_max(&P.dev->pub, hp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (hs) stop = true;
    ps_mirror(P);
    return hp > k;
}

// Copy the kernel's counters into the host's control block (lane 0).
__device__ __forceinline__ void ps_mirror(const PsParams &P) {
    PsHost *h = P.host;
    __hip_atomic_store(&h->seen_cur, __hip_atomic_load(&P.dev->cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&h->seen_pub, __hip_atomic_load(&P.dev->pub, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&h->seen_started,
                       __hip_atomic_load(&P.dev->started, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(&h->seen_peak,
                       __hip_atomic_load(&P.dev->active_peak, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(1))) void pserver_kernel(PsParams P) {
    __shared__ PsLds L;
    __shared__ PsReq R;  // the request whose units this workgroup takes (a copy of its ring slot)
    __shared__ dd vt[2 * (2 * TOR_MAX_N - 2)];
    __shared__ PsPath path;
    __shared__ long long s_k, s_u;
    __shared__ int s_act;
    const int lane = threadIdx.x;
    wave_tree_init<0>(L.top.w.ab, lane);
    dd *ws = P.scratch + (long long)blockIdx.x * P.scratch_stride;
    long long cached = -1;
    int backoff = 0;  // lane 0: log2 of the sleeps between idle polls
    unsigned int acq_gen = 0;  // newest device-data generation this workgroup has acquired
    unsigned long long idle_since = wall_clock64();
    if (lane == 0) {
        __hip_atomic_fetch_add(&P.dev->started, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned int a = __hip_atomic_fetch_add(&P.dev->active, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_max(&P.dev->active_peak, a + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // lane 0: a unit taken by a fetch-and-add that found the slot already
    // reset for a later (published) request; and whether this workgroup is
    // counted in P.dev->idle
    long long pend_k = -1, pend_u = 0;
    bool counted = false;
    for (;;) {
        // --- claim a unit (lane 0 decides; act: 0 retry, 1 unit, 2 load the
        // request, 3 exit).  Polling loads are relaxed: they only pick what to
        // do; the request's data is acquired once, when it is loaded.
        if (lane == 0) {
            int act = 0;
            bool stalled = false;  // no work to take now
            const unsigned long long k = __hip_atomic_load(&P.dev->cur, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            unsigned long long *ctl = P.dev->pubx[blockIdx.x & 7];
            const unsigned long long px = __hip_atomic_load(&ctl[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const bool closing =
                __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == P.epoch;
            const unsigned long long pub = px & ~(1ULL << 63);
            bool stop = (px >> 63) != 0;
            if (pend_k >= 0) {
                // the held unit: its request is published, so this waits at
                // most until this workgroup's copy of the control block shows it
                if ((unsigned long long)pend_k < pub) {
                    s_k = pend_k;
                    if (pend_k != cached) {
                        act = 2;
                    } else {
                        if (pend_u < R.units) {  // else an overshoot: nothing to do
                            act = 1;
                            s_u = pend_u;
                        }
                        pend_k = -1;
                    }
                } else if (stop) {
                    act = 3;
                } else if (!ps_refresh(P, k, backoff, stop)) {
                    for (int b = 0; b < (1 << backoff); ++b) __builtin_amdgcn_s_sleep(127);
                    if (backoff < kPsMaxBackoff) ++backoff;
                }
            } else if (closing || stop) {
                act = 3;  // the launch is closing (or the host stops): claim nothing more
            } else if (k < pub) {
                s_k = (long long)k;
                if ((long long)k != cached) {
                    act = 2;
                } else {
                    // one fetch-and-add claims a unit; the check before it keeps
                    // late workgroups off a finished request's counter
                    const int slot = (int)(k % TOR_PS_SLOTS);
                    const unsigned long long klo = k & 0xffffffffULL;
                    unsigned long long v0 =
                        __hip_atomic_load(&P.dev->next[slot], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const int ahead = (int)(unsigned int)((v0 >> 32) - klo);
                    if (ahead == -TOR_PS_SLOTS) {
                        // the slot still counts request k - TOR_PS_SLOTS, which
                        // is finished (k is published): reset it for k
                        __hip_atomic_compare_exchange_strong(&P.dev->next[slot], &v0, klo << 32, __ATOMIC_RELAXED,
                                                             __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    } else if (ahead > 0 || (ahead == 0 && (long long)(v0 & 0xffffffffULL) >= R.units)) {
                        ps_advance(P, k);  // every unit of k is taken
                    } else if (ahead < 0) {
                        stalled = true;  // not expected: wait as for no work
                    } else {
                        const unsigned long long v = __hip_atomic_fetch_add(&P.dev->next[slot], 1ULL,
                                                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        const long long u = (long long)(v & 0xffffffffULL);
                        const int d = (int)(unsigned int)((v >> 32) - klo);
                        if (d == 0) {
                            if (u < R.units) {
                                act = 1;
                                s_u = u;
                            } else {
                                ps_advance(P, k);  // the last unit went in between: overshoot
                            }
                        } else {
                            // k finished and the slot was reset for request
                            // k + d between the check and the add (this wave was
                            // held up): this workgroup took that request's unit u
                            pend_k = (long long)k + d;
                            pend_u = u;
                        }
                    }
                }
            } else {
                // no work.  Eight workgroups (and any at its longest backoff)
                // refresh the copies of the control block, one per refresh
                // period; the others poll their XCD's copy.
                const bool fresh = ps_refresh(P, k, backoff, stop);
                if (stop) act = 3;
                else stalled = !fresh;
            }
            if (stalled) {
                if (wall_clock64() - idle_since > (unsigned long long)P.idle_ticks) {
                    // past the idle time: counted as idle; once every running
                    // workgroup is, this one closes the launch (bounded: the
                    // kernel leaves the device as a whole)
                    if (!counted) {
                        counted = true;
                        __hip_atomic_fetch_add(&P.dev->idle, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    if (__hip_atomic_load(&P.dev->idle, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >=
                        __hip_atomic_load(&P.dev->active, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                        for (int x = 0; x < 8; ++x)
                            __hip_atomic_store(&P.dev->pubx[x][1], P.epoch, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                        __hip_atomic_store(&P.host->seen_closing, P.epoch, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_SYSTEM);
                        act = 3;
                    }
                }
                if (act != 3) {
                    // exponential backoff, up to 8 sleeps of ~3.4 us between polls:
                    // a thousand idle workgroups must not crowd the memory path
                    // the busy ones use
                    for (int b = 0; b < (1 << backoff); ++b) __builtin_amdgcn_s_sleep(127);
                    if (backoff < kPsMaxBackoff) ++backoff;
                }
            } else if (pend_k < 0) {
                backoff = 0;
            }
            if (counted && (act == 1 || act == 2 || act == 3)) {  // found work, or leaves
                counted = false;
                __hip_atomic_fetch_sub(&P.dev->idle, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            s_act = act;
        }
        wave_sync();
        const int act = s_act;
        if (act == 3) break;
        if (act == 0) continue;
        if (act == 2) {
            // copy request s_k from its ring slot (host memory) into LDS, then
            // acquire what the host wrote to device memory before publishing it
            // (once per generation of device data)
            const long long k = s_k;
            const unsigned long long *src =
                reinterpret_cast<const unsigned long long *>(&P.ring[k % TOR_PS_SLOTS]);
            unsigned long long *dst = reinterpret_cast<unsigned long long *>(&R);
            constexpr int W = (int)(sizeof(PsReq) / 8);
            static_assert(sizeof(PsReq) % 8 == 0, "request copied in 8-byte words");
            for (int w = lane; w < W; w += 64)
                dst[w] = __hip_atomic_load(&src[w], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            wave_sync();
            if (R.gen != acq_gen) {  // device data made since this workgroup last acquired
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                acq_gen = R.gen;
            }
            wave_sync();
            const bool ok = R.seq == k;
            cached = ok ? k : -1;
            if (!ok && lane == 0) {
                if (R.seq > k) {  // the slot already holds a later request: k is finished
                    unsigned long long kk = (unsigned long long)k;
                    __hip_atomic_compare_exchange_strong(&P.dev->cur, &kk, kk + 1, __ATOMIC_RELAXED,
                                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                } else {
                    __builtin_amdgcn_s_sleep(64);  // not visible yet (the claim loop still sees the stop flag)
                }
            }
            wave_sync();
            continue;
        }
        // --- a unit of request cached
        idle_since = wall_clock64();
        const long long u = s_u;
        if (R.type == TOR_PS_PROB) ps_prob_unit(R, u, ws, L, vt, path, lane);
        else ps_chain_unit(R.cp, (int)u, L.chain, lane);
        // every lane's results (task partials in device memory, chain outputs in
        // host memory) before the unit is counted
        if (R.type == TOR_PS_PROB) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        wave_sync();
        if (lane == 0) {
            const int slot = (int)(R.seq % TOR_PS_SLOTS);
            const unsigned int old =
                __hip_atomic_fetch_add(&P.dev->done[slot], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            s_act = (long long)old + 1 == R.units ? 1 : 0;
        }
        wave_sync();
        if (s_act) {  // the last unit: finish the request
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            wave_sync();
            if (R.type == TOR_PS_PROB) {
                const Partial res = ps_reduce(R, L, lane);
                if (lane == 0) ps_publish(P, R, &res);
            } else if (lane == 0) {
                ps_publish(P, R, nullptr);
            }
        }
        wave_sync();
    }
    if (lane == 0 && __hip_atomic_fetch_sub(&P.dev->active, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 1)
        ps_mirror(P);  // the last workgroup to exit
}

}  // namespace tor

hipError_t tor_launch_pserver(const PsParams &P, int grid, hipStream_t st) {
    if (grid < 1) return hipErrorInvalidValue;
    (void)hipGetLastError();  // report only this launch's error
    hipLaunchKernelGGL(tor::pserver_kernel, dim3((unsigned)grid), dim3(64), 0, st, P);
    return hipGetLastError();
}

int tor_pserver_occupancy(int device) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, tor::pserver_kernel, 64, 0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return per_cu * cus;
}
