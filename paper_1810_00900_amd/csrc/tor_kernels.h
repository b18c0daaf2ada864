// Internal launch interface between the host library and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define TOR_MAX_N 32
// largest wave-tier task (modes per task): nine-mode trees, plus 10- and
// 11-mode tasks that take their top one or two decisions in LDS first
#define TOR_TASK_MAX 11

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

// Work lists of the batched launches.  Several queries (each its own subset
// tree) share one launch; each job is one query's share, and a block finds its
// job from its flat index, so the work done for a query never depends on the
// other queries in the launch.

// expansion of level d of one query: 2^d parent nodes with r modes
struct ExpandJob {
    const NodeDesc *par;
    NodeDesc *chi;
    unsigned long long child_base;
    int r;
    int d;  // 1: displaced state, the packed matrix has the mean row first
};

// wave-tier tasks of one query: tasks[0 .. count) -> out[0 .. count); the
// flat task index of tasks[0] is `begin` (jobs sorted by begin)
struct WaveJob {
    const NodeDesc *tasks;
    Partial *out;
    long long begin;
};

// one reduction stage of one query: in[0 .. count) -> out[0 .. ceil(count/chunk))
struct ReduceJob {
    const Partial *in;
    Partial *out;
    long long count;
    long long block_begin;
};

#define TOR_REDUCE_CHUNK 1024

// Single-launch subset sum of a small zero-mean tree (tor_fused.hip): the tree
// of n <= TOR_FUSED_MAX_N modes with J-mode wave-tier tasks is cut into 2^g
// units of 2^t consecutive tasks (n = g + t + J, t <= TOR_FUSED_TMAX); flat
// unit index `begin` is the tree's first (jobs sorted by begin).  part holds
// 2^(g + t) task partials followed by the first reduction stage's block sums;
// ctr holds 1 + (number of blocks) completion counters, zero before the
// launch and zero again after it; res receives the tree's (T, A) and may be
// host memory.
#define TOR_FUSED_MAX_N 22
#define TOR_FUSED_TMAX 4
struct FusedJob {
    const void *root;  // Sigma_C, packed lower, EN(n) scalars
    Partial *part;
    unsigned *ctr;
    Partial *res;
    long long begin;
    int n, g, t;
};

// Job count and total work of a launch whose plan was made on the device
// (stream-ordered batches): the kernels read them at entry when given a
// non-null pointer, instead of their by-value arguments.
struct LaunchDims {
    long long njobs;
    long long total;
};

// one vacuum-conditioning step of one query: its packed matrix of r modes (the
// no-click modes last) loses its last mode in place; acc = {P_vac hi, lo,
// log P_vac} of the modes conditioned so far
struct CondJob {
    dd *mat;
    double *acc;
    double *qout;     // if not null: this step's pivot factor q (hi, lo)
    long long begin;  // first block of the launch that works on this job
    int r;
    int d;            // 1: displaced state, the packed matrix has the mean row first
};

// Blocked conditioning: b <= TOR_COND_BLOCK no-click modes of one query per
// pair of launches.  The panel launch walks the b modes in order on the
// pivot block and, per column x of the rest, records each step's two scaled
// pivot columns V[(2t + w) ld + x]; the bulk launch then applies the b
// rank-2 updates to every remaining entry in step order (the per-mode
// kernel's operations, entry for entry).
#define TOR_COND_BLOCK 16
struct CondBlockJob {
    dd *mat;                 // packed matrix, R = 2r + d rows before the block
    dd *V;                   // [2b][ld]: the block's scaled pivot columns
    double *acc;             // (p hi, p lo, log p), updated in step order
    long long begin_panel;   // first workgroup of the panel launch for this job
    long long begin_bulk;    // first workgroup of the bulk launch for this job
    int r, b, d, ld;
    int passes;              // panel: column groups per workgroup (its block steps serve all of them)
};
hipError_t tor_launch_cond_panel(const CondBlockJob *jobs, int njobs, long long total_blocks, hipStream_t st);
hipError_t tor_launch_cond_bulk(const CondBlockJob *jobs, int njobs, long long total_blocks, hipStream_t st);
// workgroups of a job's panel (passes x 256 / TOR_COND_TPC columns each) and bulk (32 x 32 tiles) launches
#define TOR_COND_TPC 16 // panel kernel: threads per column (256 / TOR_COND_TPC columns per workgroup)
__host__ __device__ inline long long cond_panel_blocks(int r, int b, int d, int passes) {
    const long long rb = 2LL * (r - b) + d, per = (long long)(256 / TOR_COND_TPC) * passes;
    return rb > 0 ? (rb + per - 1) / per : 1;
}
__host__ __device__ inline long long cond_bulk_blocks(int r, int b, int d) {
    const long long rb = 2LL * (r - b) + d, t = (rb + 31) / 32;
    return t > 0 ? t * (t + 1) / 2 : 0;
}

#define TOR_COND_CHUNK 1024
// largest matrix (modes) a conditioning step takes: its two scaled pivot
// columns (2 * (2r - 2) double-doubles) must fit 64 KiB of LDS
#define TOR_COND_MAX_MODES 1024

// ---------------------------------------------------------------- stream-ordered batches
// A batch whose click patterns live in device memory is planned on the device
// (tor_async.hip): the same per-query trees, job tables and reduction order as
// the host planner, built by one workgroup with deterministic block scans.

#define TOR_ASYNC_STAGES 4   // reduction stages (TOR_REDUCE_CHUNK^4 tasks)

struct AsyncQuery {
    int status;          // tor_status of this query
    int n, J, G;         // clicks, task size, HBM levels
    long long nt;        // tasks (2^G; 0 when n = 0)
    long long entries;   // pool scalars of the tree
    long long pb;        // reduction-stage partials
    long long pool_off, desc_off, pb_off;
    long long final_off; // partial holding the sum: partA (final_buf 0) or partB (1)
    int final_buf;
    int nstage;
    double log_det;      // log det Sigma_C (binary64 Cholesky)
    double quad;         // displaced states: mu_C^T Sigma_C^-1 mu_C, or h_C^T G^-1 h_C for the
                         // information form (binary64); else 0
    int jac;             // full pattern on an inverted state: the tree sums G = sigma_Q^-1 over C
    double jscale;       // jac: (-1)^n det(G)^1/2 (times exp(-quad / 2) when displaced, binary64),
                         // T(Sigma_C) = jscale T(G)
    double log_pvac;     // jac: log P_vac(N) = -(log det sigma_Q + log det G) / 2 (displaced:
                         // - mu^T sigma_Q^-1 mu / 2 + quad / 2); else 0
    long long slot;      // planner scratch: position of the query's job in a table
    int C[TOR_MAX_N];    // clicked modes, ascending
};

struct AsyncPlan {
    int nq, m, is_dd, gcap, jmax;
    int D;               // 1: displaced state (mean row first in every packed matrix)
    const double *mean;  // displaced states: device copy of the mean (2m), else null
    const void *inv;     // inverted state: sigma_Q^-1 packed lower, double-double words; else null
    const void *inv_h;   // inverted displaced state: h = sigma_Q^-1 mu (2m double-double words); else null
    // inverted state: det(sigma_Q)^-1/2 (times exp(-mu^T sigma_Q^-1 mu / 2) when displaced),
    // log det sigma_Q and mu^T sigma_Q^-1 mu
    double det_rsqrt_hi, det_rsqrt_lo, log_det_sigq, mu_k_mu;
    double inv_cond_u;   // inverted state: elimination roundoff carried by G (m u of the inverse)
    int nkinds;          // tree kinds in the batch: 2 when full patterns of an inverted displaced
                         // state (information form, kind 1) join the displaced trees (kind 0)
    int J_of_n[TOR_MAX_N + 1];
    long long pool_cap, desc_cap, pb_cap;  // capacities (scalars, descriptors, partials)
    AsyncQuery *q;
    void *pool;
    NodeDesc *roots, *descA, *descB;
    Partial *partA, *partB;
    ExpandJob *exp_jobs;   // [nkinds][gcap][nq]
    WaveJob *wave_jobs;    // [nkinds][TOR_TASK_MAX + 1][nq]
    ReduceJob *red_jobs;   // [TOR_ASYNC_STAGES][nq]
    LaunchDims *dims;      // per kind: expand [gcap], wave [TOR_TASK_MAX + 1]; then reduce [TOR_ASYNC_STAGES]
};

hipError_t tor_launch_async_prologue(const int8_t *d_patterns, const double *d_cov, const AsyncPlan &P,
                                     hipStream_t st);
hipError_t tor_launch_async_finalize(const AsyncPlan &P, double tol, int prec_used, void *d_out, hipStream_t st);

// Launchers.  With dyn != nullptr (a plan made on the device) the kernels read
// the job count and total work from dyn, and the host-side grid argument
// (grid_cap, total_blocks) is the grid itself, a bound on the work.
// disp = 1: displaced state (every packed matrix has the mean row first);
// disp = -1: the information form of a displaced state's full patterns.
hipError_t tor_launch_wave(int is_dd, int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                           int grid_cap, hipStream_t st, const LaunchDims *dyn = nullptr, int disp = 0);
hipError_t tor_launch_wave_disp(int is_dd, int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                                int grid_cap, hipStream_t st, const LaunchDims *dyn);
// disp = -1: the information form (first row sigma_Q^-1 mu, pivots carry exp(+|w|^2 / 2))
hipError_t tor_launch_wave_info(int is_dd, int J, const WaveJob *jobs, int njobs, long long total, const void *pool,
                                int grid_cap, hipStream_t st, const LaunchDims *dyn);
hipError_t tor_launch_expand(int is_dd, const ExpandJob *jobs, int njobs, int log2npar, void *pool, int grid_cap,
                             hipStream_t st, const LaunchDims *dyn = nullptr, int disp = 0);
hipError_t tor_launch_reduce(const ReduceJob *jobs, int njobs, long long total_blocks, hipStream_t st,
                             const LaunchDims *dyn = nullptr);
hipError_t tor_launch_gather(const Partial *const *src, int n, Partial *dst, hipStream_t st);
// ws: grid * ws_stride scalars of per-workgroup scratch (ws_stride >= (1 + t) EN(J + t)
// for every job); J in 1..11.
hipError_t tor_launch_fused(int is_dd, int J, const FusedJob *jobs, int njobs, long long units, void *ws,
                            long long ws_stride, int grid, hipStream_t st);
hipError_t tor_launch_condition(const CondJob *jobs, int njobs, long long total_blocks, int rmax, hipStream_t st);

// ---- quad-double term tier (one tree per launch sequence)
// Pool layout: every node slot is [path coefficient (one qd)][packed matrix],
// a descriptor's off points at the matrix, so the coefficient is pool[off - 1]
// (the exclude child shares its parent's slot and coefficient).
#define TOR_QD_TASK_MAX 8  // modes per wave-tier task (two-mode register leaf)

struct PartialQ {
    double t0, t1, t2, t3, a, pad0, pad1, pad2;
};

struct ReduceJobQ {
    const PartialQ *in;
    PartialQ *out;
    long long count;
    long long block_begin;
};

// one vacuum-conditioning step of one query in quad-double: mat (r modes,
// packed lower) loses its last mode; cols is scratch for the two scaled pivot
// columns (2 (2r - 2) words); acc as in CondJob.
struct CondJobQ {
    void *mat;
    double *acc;
    void *cols;
    double *qout;  // if not null: this step's pivot factor q (double-double rounding, hi, lo)
    long long begin;
    int r;
    int d;  // 1: displaced state, the packed matrix has the mean row first
};

hipError_t tor_launch_wave_qd(int J, const WaveJob *jobs, int njobs, long long total, const void *pool, int grid_cap,
                              hipStream_t st, int disp = 0);
hipError_t tor_launch_expand_qd(const ExpandJob *jobs, int njobs, int log2npar, void *pool, int grid_cap,
                                hipStream_t st, int disp = 0);
hipError_t tor_launch_reduce_qd(const ReduceJobQ *jobs, int njobs, long long total_blocks, hipStream_t st);
// one conditioning step: the pivot columns of every job, then the update
hipError_t tor_launch_condition_qd(const CondJobQ *jobs, int njobs, long long total_blocks, hipStream_t st);

// ---- chain-rule sampler
#define TOR_CHAIN_MAX 16      // step-tree cap of the compact sampler kernel (clicks so far + 1)
#define TOR_CHAIN_MAX_BIG 21  // step-tree cap of the large sampler kernel (up to 20 clicks)

struct ChainParams {
    const double *K;                 // K_j, full row-major (2j+2)^2, concatenated
    const unsigned long long *koff;  // offset of K_j in K
    const double *H;                 // displaced states: h_j = K_j mu[0..2j+1], concatenated (else null)
    const unsigned long long *hoff;  // offset of h_j in H
    const double *Klo;               // double-double terms: low words of K (and of H), else null
    const double *Hlo;
    int m;
    int n_post;                      // < 0: no postselection
    int cap;                         // most clicks a chain may carry (<= TOR_CHAIN_MAX_BIG - 1)
    unsigned long long seed;
    long long chain_begin;
    int nchains;
    unsigned char *outcome;          // nchains x m (0/1; 0 after a stop)
    signed char *status;             // nchains: 1 accepted, 0 rejected, 2 exceeded the tree cap
    double *trace_p;                 // optional nchains x m: P(click) (NaN where not evaluated)
    double *trace_u;                 // optional nchains x m: uniform draw
    double *subsets;                 // optional nchains: subset terms evaluated
    double *trace_r;                 // optional nchains x m: cancellation ratio max(A0/|X0|, A1/|X1|)
    double *trace_b;                 // optional nchains x m: bound on the absolute error of P(click)
};

hipError_t tor_launch_chains(const ChainParams &P, int grid_cap, hipStream_t st);

// ---- persistent request loop (tor_pserver.hip)
// Requests are published in order into a ring of TOR_PS_SLOTS slots in
// host-coherent memory; request k uses slot k % TOR_PS_SLOTS.  Workgroups of
// the persistent kernel claim the units of the request being distributed with
// a fetch-and-add on the slot's counter, which carries the request's sequence
// number in its high word.  A check before the add keeps workgroups off a
// finished request's counter, and a slot's counter is reset for its next
// request only once that request is published, by the first workgroup that
// reaches it; so a workgroup held up between the check and the add either
// overshoots the old request or takes a unit of the published one.  No unit
// waits for another: the last unit of a request (counted per slot) reduces and
// publishes its result.  The kernel leaves the device as a whole: when every
// running workgroup has been without work for the idle time, one of them
// closes the launch and all exit (each after the unit it holds); the host
// launches it again when work arrives.
#define TOR_PS_SLOTS 4096
#define TOR_PS_LMAX 8  // most depth-first levels a probability unit walks
#define TOR_PS_TASK_MAX TOR_TASK_MAX  // the persistent kernel takes every task size

enum { TOR_PS_PROB = 1, TOR_PS_CHAINS = 2 };

struct PsReq {             // host-coherent; the host writes every field, then seq, then publishes
    long long seq;         // request index
    int type;              // TOR_PS_PROB or TOR_PS_CHAINS
    unsigned int gen;      // generation of the device data the request reads (acquired when new)
    int n, J, g;           // probability: clicks, task modes (<= n), unit depth (units = 2^g)
    int t;                 // probability: depth-first levels of a unit (tasks per unit = 2^t)
    int m, jac;            // modes of the state; 1: gather G from the inverse (a full pattern)
    long long units;       // work units of the request
    long long tasks;       // probability: wave tasks, 2^(g + t)
    const double *cov;     // device: the state's covariance, 2m x 2m row-major (jac = 0)
    const dd *inv;         // device: the state's inverse, packed lower, double-double words (jac = 1)
    Partial *part;         // device: task partials, then the reduction stages
    ChainParams cp;        // chains: parameters of chains cp.chain_begin .. + units (outputs host-coherent)
    int C[TOR_MAX_N];      // probability: clicked modes, ascending
};

struct PsResult {          // host-coherent, one per slot
    unsigned long long done;  // seq + 1 once the request is complete
    double t_hi, t_lo, a;     // probability: the subset sum T and the sum of |terms|
};

struct PsHost {            // host-coherent control block
    unsigned long long published;  // requests 0 .. published - 1 are in the ring
    unsigned int stop;             // 1: the kernel exits once it has no work
    unsigned int pad;
    // written by the kernel (on refresh and when its last workgroup exits), for
    // the host's statistics without a device copy
    unsigned long long seen_cur, seen_pub;
    unsigned int seen_started, seen_peak;
    unsigned long long seen_closing;  // the newest launch that decided to close
};

struct PsDev {             // device memory (zeroed, next[s] = s << 32, before the first launch)
    unsigned long long cur;        // request whose units are being claimed
    unsigned long long pub;        // the kernel's copy of PsHost::published
    unsigned long long refresh;    // wall-clock time of the last copy of the control block
    unsigned int idle;             // running workgroups past the idle time without work
    unsigned int active;           // workgroups of the kernel running now
    unsigned int started;          // workgroups that have started (all launches)
    unsigned int active_peak;      // most workgroups running at once
    // copies of the control words, one per XCD (workgroup i polls copy i % 8,
    // each in a line of its own): [0] pub with the host's stop flag in bit 63,
    // [1] the launch (PsParams::epoch) that is closing
    unsigned long long pubx[8][16];
    unsigned long long next[TOR_PS_SLOTS];  // (seq << 32) | next unit of the slot's request (seq's low word)
    unsigned int done[TOR_PS_SLOTS];        // finished units of the slot's request
};

struct PsParams {
    PsHost *host;
    PsReq *ring;                // [TOR_PS_SLOTS]
    PsResult *res;              // [TOR_PS_SLOTS]
    PsDev *dev;
    dd *scratch;                // per-workgroup buffers of the depth-first walk
    long long scratch_stride;   // double-double words per workgroup
    long long idle_ticks;       // the launch closes after every workgroup has been this long without work
    long long refresh_ticks;    // the control block is read at most this often
    unsigned long long epoch;   // launch number (from 1)
};

// words of per-workgroup scratch: the unit's node and one buffer per level
#define TOR_PS_SCRATCH_WORDS ((1 + TOR_PS_LMAX) * (TOR_MAX_N * (2 * TOR_MAX_N + 1)))

hipError_t tor_launch_pserver(const PsParams &P, int grid, hipStream_t st);
// workgroups of the persistent kernel that fit the device at once
int tor_pserver_occupancy(int device);

