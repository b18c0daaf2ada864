"""Benchmark: large single Torontonians on an 800-mode GBS state.

One step = one call of tor_probability (the whole hot path: sigma_Q, reduction
of the click pattern to Sigma_C, the subset-tree kernels, the double-double
reduction and the final assembly) for a marginal click pattern with n clicks
(default n = 28, 2^28 subset terms) of the 800-mode state (Haar U,
r_i ~ U[0.3, 0.9], seed 50), double-double terms (the precision tier that meets
the 1e-8 target at these sizes).

Printed: one JSON line with the subset-determinant rate, the roofline of the
dominant (wave-tier) kernel from HIP events on the library's stream, and the
CPU oracle timed on a bounded sample of the same sum.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--n 28]
"""
import argparse
import collections
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 subset-dets/sec + % FP64 peak at n=20–28; p50/p99 query latency"
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector peak (256 CU x 128 flop/clk x 2.4 GHz)


# ---------------------------------------------------------------------------
# Algorithmic flop count of the double-double subset tree (FMA = 2 flops),
# from the operation counts of the dd primitives (csrc/dd.hpp).
# ---------------------------------------------------------------------------
F_TWO_SUM, F_FAST_TWO_SUM, F_TWO_PROD = 6, 3, 3
F_DD_ADD = 2 * F_TWO_SUM + 1 + F_FAST_TWO_SUM + 1 + F_FAST_TWO_SUM          # 20
F_DD_MUL = F_TWO_PROD + 1 + 2 + 1 + F_FAST_TWO_SUM                          # 10
F_DD_SUB_DOT2 = 2 * F_TWO_PROD + 2 * 3 + 2 * F_TWO_SUM + 6 + F_TWO_SUM      # 36
F_DD_DET2 = 2 * F_TWO_PROD + 3 + 2 + F_TWO_SUM + 4 + F_TWO_SUM              # 27
F_DD_RSQRT = 2 + 2 * F_TWO_PROD + 4 + 2 + 2 + F_FAST_TWO_SUM                # 19


def E(r):
    return r * (2 * r + 1)


def dd_node_flops(r):
    """Flops to expand one r-mode node (r >= 2) into its include child and to
    combine T, A; r == 1: a leaf pivot."""
    if r == 1:
        return F_DD_DET2 + F_DD_RSQRT + F_DD_ADD + 1
    piv = 2 * F_DD_RSQRT + 3 * F_DD_MUL + (F_DD_MUL + F_DD_ADD)
    cols = 2 * (r - 1) * (3 * F_DD_MUL + F_DD_ADD)
    ents = E(r - 1) * F_DD_SUB_DOT2
    comb = F_DD_MUL + F_DD_ADD + 2
    return piv + cols + ents + comb


def tree_flops(n, top=None):
    """Flops of the full subset tree of n modes; with top = J only the part
    below the nodes of J modes (what one wave-tier task does), per task."""
    r0 = n if top is None else top
    # a node with r modes has 2^(r0 - r) copies below the start
    return sum((2 ** (r0 - r)) * dd_node_flops(r) for r in range(1, r0 + 1))


def wave_kernel_name(prec, J, D=0):
    """Name of the wave-tier kernel that runs J-mode tasks (as rocprofv3 lists
    it, template arguments <scalar, task modes, mean rows> without spaces)."""
    s = "dd" if prec == "dd" else "double"
    return f"wave_kernel_top<{s},{J},{D}>" if J > 9 else f"wave_kernel<{s},{J},{D}>"


def kernel_slug(kernel):
    """File-name form of a wave-kernel name: wave_kernel_top<dd,10,0> ->
    wave_kernel_top_dd10 (a displaced kernel gets the suffix _disp),
    wave_kernel_qd<8,0> -> wave_kernel_qd8."""
    base, args = kernel[:-1].split("<")
    parts = args.split(",")
    if len(parts) == 2:  # quad-double: <J,D>
        return f"{base}{parts[0]}" + ("_disp" if parts[1] == "1" else "")
    s, J, D = parts
    return f"{base}_{'f64' if s == 'double' else s}{J}" + ("_disp" if D == "1" else "")


def cpu_baseline(cov, pattern, n, seconds_target=15.0):
    """Time the binary128 oracle on a strided sample of the same subset sum."""
    import oracle
    threads = oracle.num_threads()
    count = 2048
    # grow the sample until it takes ~1 s, then size it for the target
    while True:
        stride = max(1, (2 ** n) // count) | 1
        t = time.perf_counter()
        oracle.formS_range(cov, pattern, 0, stride, count)
        dt = time.perf_counter() - t
        if dt > 1.0 or count >= 2 ** n:
            break
        count *= 4
    count = int(min(2 ** n, count * max(1.0, seconds_target / dt)))
    stride = max(1, (2 ** n) // count) | 1
    t = time.perf_counter()
    oracle.formS_range(cov, pattern, 0, stride, count)
    dt = time.perf_counter() - t
    # the same oracle on one thread, a sample sized for about 5 s (masks 1 + j * stride1)
    count1 = max(1, int(count / dt / max(1, threads) * 5.0))
    stride1 = max(1, (2 ** n) // count1) | 1
    t = time.perf_counter()
    oracle.formS_range(cov, pattern, 1, stride1, count1, threads=1)
    dt1 = time.perf_counter() - t
    return {"value": count / dt, "unit": "subset-dets/s", "cores": threads, "kind": "oracle",
            "sample": f"{count} of the 2^{n} subsets (masks 0, {stride}, 2*{stride}, ... mod 2^{n}) of the "
                      f"same n={n} sum, binary128 Cholesky per subset, {dt:.1f} s",
            "single_thread": {"value": count1 / dt1, "unit": "subset-dets/s", "cores": 1,
                              "sample": f"{count1} subsets (masks 1 + j*{stride1}), {dt1:.1f} s"}}


KERNEL_SOURCES = ["paper_1810_00900_amd/csrc/dd.hpp", "paper_1810_00900_amd/csrc/qd.hpp",
                  "paper_1810_00900_amd/csrc/tor_tree.hpp", "paper_1810_00900_amd/csrc/tor_wave.hpp",
                  "paper_1810_00900_amd/csrc/tor_kernels.hip", "paper_1810_00900_amd/csrc/tor_kernels_disp.hip",
                  "paper_1810_00900_amd/csrc/tor_kernels_info.hip", "paper_1810_00900_amd/csrc/tor_kernels_qd.hip",
                  "paper_1810_00900_amd/csrc/tor_kernels.h"]


def measured_fp64(kernel, kernel_ms):
    """Executed FP64 rate of the wave-tier kernel from the committed rocprofv3
    PMC pass (SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 per launch, 64 lanes per
    wave instruction, FMA = 2 flops) over this run's kernel time; None when
    the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"pmc_fp64_{kernel_slug(kernel)}_m800_n28.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    if d.get("sources_sha256") != h.hexdigest() or d.get("kernel") != kernel:
        return None
    flops = d["executed_fp64_flops_per_launch"]
    tf = flops / (kernel_ms * 1e-3) / 1e12
    return {"executed_flops_per_launch": flops, "achieved": tf, "frac": tf / FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "basis": "executed FP64 VALU instructions x 64 lanes (FMA = 2)"}


def measured_traffic(kernel):
    """HBM bytes per launch of the wave-tier kernel from the committed
    rocprofv3 FETCH_SIZE/WRITE_SIZE measurement (profiles/), scaled by the
    copy-kernel calibration; None when the kernel sources changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_slug(kernel)}_m800_n28.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    h = hashlib.sha256()
    for s in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    if d.get("sources_sha256") != h.hexdigest() or d.get("kernel") != kernel:
        return None
    return d["traffic_bytes_per_launch"]


def copy_calibration():
    """A plain 1 GiB device copy, profiled with the same counters to scale
    FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch
    n = 1 << 27
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": n * 8}))


def per_n_rates(ctx, cov, prec, ns=(20, 24, 28, 32), full=False, mean=None):
    """subset-dets/s of single Torontonians at several n (whole calls).  With
    full=True every other mode is a no-click mode (the full-pattern variant:
    the same tree after conditioning on the m - n no-click modes).  With a
    mean vector the state is displaced (tor_probability_displaced)."""
    import gbs_inputs as gi
    out = {}

    def call(pat):
        if mean is None:
            return ctx.probability(cov, pat, prec=prec, tol=1e-8)
        return ctx.probability_displaced(cov, mean, pat, prec=prec, tol=1e-8)

    for n in ns:
        pat = gi.config5_pattern(n).copy()
        if full:
            pat[pat == -1] = 0
        reps = 1 if n >= 32 else 3
        call(pat)
        ctx.reset_stats()
        t = time.perf_counter()
        for _ in range(reps):
            r = call(pat)
        dt = (time.perf_counter() - t) / reps
        st = ctx.stats()
        kms = (st["wave_ms"] + st["expand_ms"] + st["reduce_ms"]) / reps
        out[str(n)] = {"subset_dets_per_s": 2.0 ** n / dt, "ms": dt * 1e3, "kernel_ms": kms,
                       "rel_err_bound": r.rel_err_bound}
        if prec == "dd" and mean is None and not full:
            # algorithmic flops of the whole tree (expand levels and wave tasks)
            # over the whole call and over the kernels' time, against FP64 peak
            f = tree_flops(n)
            out[str(n)]["frac_call"] = f / dt / 1e12 / FP64_PEAK_TFLOPS
            out[str(n)]["frac_kernels"] = f / (kms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS if kms > 0 else None
        if full:
            out[str(n)]["no_click_modes"] = int((pat == 0).sum())
            out[str(n)]["condition_launches"] = st["condition_launches"] // reps
    return out


def batch_rate(ctx, cov, n, nq, reps=5, seed=60):
    """Throughput of nq marginal n-click queries (distinct random click sets
    on the state) in one tor_batch call, double-double terms: subset-dets/s
    and the algorithmic FP64 fraction over the whole call."""
    import numpy as np
    rng = np.random.default_rng(seed)
    m = cov.shape[0] // 2
    pats = np.full((nq, m), -1, np.int8)
    for q in range(nq):
        pats[q, rng.choice(m, n, replace=False)] = 1
    st = ctx.state(cov)
    ctx.batch(st, pats, prec="dd", tol=1e-8)
    t = time.perf_counter()
    for _ in range(reps):
        ctx.batch(st, pats, prec="dd", tol=1e-8)
    dt = (time.perf_counter() - t) / reps
    st.close()
    return {"queries": nq, "ms_per_call": dt * 1e3, "subset_dets_per_s": nq * 2.0 ** n / dt,
            "frac_call": nq * tree_flops(n) / dt / 1e12 / FP64_PEAK_TFLOPS}


def full_pattern_inverse(ctx, cov, ns=(20, 28), mean=None):
    """Full patterns (the per_n_full_pattern queries) on a state inverted once
    (tor_state_invert): the time of the inversion per precision, then each
    query as a one-query tor_batch on that state (a gather of sigma_Q^-1 over
    the clicked modes and one subset tree, no per-query conditioning).  One
    untimed inversion per precision first takes the process's one-time kernel
    loading; each timed inversion is on a fresh state (its first device copy
    of sigma included)."""
    import gbs_inputs as gi
    out = {}
    for prec in (("dd", "qd") if mean is None else ("dd",)):
        warm = ctx.state(cov, mean=mean)
        warm.invert(prec)
        warm.close()
        st = ctx.state(cov, mean=mean)
        t = time.perf_counter()
        st.invert(prec)
        inv_ms = (time.perf_counter() - t) * 1e3
        rec = {"invert_ms": inv_ms}
        for n in ns:
            pat = gi.config5_pattern(n).copy()
            pat[pat == -1] = 0
            ctx.batch(st, pat[None, :], prec=prec, tol=1e-8)
            reps = 3
            t = time.perf_counter()
            for _ in range(reps):
                r, _ = ctx.batch(st, pat[None, :], prec=prec, tol=1e-8)
            dt = (time.perf_counter() - t) / reps
            rec[str(n)] = {"ms": dt * 1e3, "subset_dets_per_s": 2.0 ** n / dt, "rel_err_bound": r[0].rel_err_bound,
                           "no_click_modes": int((pat == 0).sum())}
        out[prec] = rec
        st.close()
    return out


def serving_full_patterns(ctx, nq=2000, workers=2):
    """Full patterns (every mode observed, n ~ U{8..20} clicks) of one 800-mode
    state served closed-loop, once on the inverted state (a gather of
    sigma_Q^-1 per query) and once with per-query conditioning (780-792
    in-place steps per query, batched by the server).  Such patterns cancel
    beyond double-double (R ~ 1e14-1e30): the results' statuses are counted,
    and the inverted-state run repeats the results whose bound exceeds tol
    with quad-double terms (a quad-double inverse of the same state), so that
    usable_queries_per_s counts every query with a result within tol."""
    import numpy as np

    import gbs_inputs as gi
    import paper_1810_00900_amd as tg
    cov = gi.state_m800(30)
    rng = np.random.default_rng(36)
    pats = [gi.full_pattern(800, gi.random_click_set(800, int(n), rng)) for n in rng.integers(8, 21, nq)]
    out = {"workload": f"{nq} full patterns, n ~ U{{8..20}}, state m=800 (seed 30), queries seed 36, dd terms, "
                       f"tol 1e-10"}
    for label, inverted in (("inverted_state", True), ("per_query_conditioning", False)):
        st = ctx.state(cov)
        t = time.perf_counter()
        if inverted:
            st.invert("dd")
        prep = time.perf_counter() - t
        srv = tg.Server(ctx, workers=workers, prec="dd", tol=1e-10, max_batch=4096)
        t0 = time.perf_counter()
        tickets = [srv.submit(st, p) for p in pats]
        res = [srv.wait(tk) for tk in tickets]
        T = time.perf_counter() - t0
        srv.stop()
        lat = np.array([x[1] for x in res])
        warn = [i for i, x in enumerate(res) if x[0].status == tg.TOR_WARN_PRECISION]
        o = {"queries_per_s": nq / T, "p50_ms": float(np.percentile(lat, 50) * 1e3),
             "p99_ms": float(np.percentile(lat, 99) * 1e3), "state_prep_ms": prep * 1e3,
             "status_ok": sum(1 for x in res if x[0].status == tg.TOR_OK), "status_warn_precision": len(warn)}
        if inverted and warn:
            sq = ctx.state(cov)
            t1 = time.perf_counter()
            sq.invert("qd")
            qprep = time.perf_counter() - t1
            t1 = time.perf_counter()
            esc, _ = ctx.batch(sq, np.stack([pats[i] for i in warn]), prec="qd", tol=1e-10)
            Tq = time.perf_counter() - t1
            sq.close()
            ok_after = o["status_ok"] + sum(1 for r in esc if r.status == tg.TOR_OK)
            o["escalated_to_qd"] = {"queries": len(warn), "seconds": Tq, "qd_inverse_ms": qprep * 1e3,
                                    "status_ok_after": ok_after,
                                    "largest_qd_bound": float(max(r.rel_err_bound for r in esc))}
            o["usable_queries_per_s"] = ok_after / (T + Tq)
        else:
            o["usable_queries_per_s"] = o["status_ok"] / T
        st.close()
        out[label] = o
    return out


def paper_worst_case(ctx, sizes=((10, 200), (12, 288), (14, 392), (16, 512), (18, 648), (20, 800)), prec="dd"):
    """The paper's runtime study, worst case (Sec. III): one sample with fixed
    outcomes, l = 2 m^2 modes, 8 dB squeezing on every mode, Haar
    interferometer, all m clicks in the first m measured modes (modes are
    measured from the last down).  Times the whole gbs_chain_fixed call."""
    import numpy as np
    import gbs_inputs as gi
    r8 = 8.0 / (20.0 * np.log10(np.e))
    out = {}
    for m, l in sizes:
        rng = np.random.default_rng([60, m])
        cov = gi.gbs_covariance(gi.haar_unitary(l, rng), np.full(l, r8))
        pat = np.zeros(l, np.int8)
        pat[l - m:] = 1
        ctx.reset_stats()
        t = time.perf_counter()
        tot, steps = ctx.chain_fixed(cov, pat, prec=prec)
        dt = time.perf_counter() - t
        st = ctx.stats()
        out[f"{l},{m}"] = {"seconds": dt, "modes": l, "clicks": m, "p": tot.p, "log_p": tot.log_p,
                           "steps": int(l), "condition_launches": st["condition_launches"],
                           "subsets": st["subsets"], "max_rel_err_bound": tot.rel_err_bound,
                           "max_cancel_ratio": tot.cancel_ratio}
    return out


def dense_subgraph(ctx, n=200, p=0.5, clique=20, k=20, target_clicks=16.0, etas=(1.0, 0.5, 0.25),
                   n_samples=500, seed=40, raw_chains=2000):
    """Dense-subgraph search with GBS (Sec. IV), synthetic graph: G(n, p) with
    a planted clique, encoded at the scale giving target_clicks mean clicks
    without loss, then uniform loss eta.  At each eta: n_samples samples
    postselected on k clicks (the search for the densest k-subgraph keeps the
    densest sample so far) against uniform random k-subsets, how many clicked
    vertices lie in the clique, raw (unpostselected) chains with the click
    cap, and the single-vertex click probabilities inside and outside the
    clique (exact marginals)."""
    import math
    import numpy as np
    import gbs_inputs as gi
    import paper_1810_00900_amd as tg
    A, cl = gi.planted_clique_graph(n, p, clique, seed)
    inside = np.zeros(n, bool)
    inside[cl] = True
    single = -np.ones((n, n), np.int8)
    np.fill_diagonal(single, 1)

    def marginals(cov):
        st = ctx.state(cov)
        res, _ = ctx.batch(st, single, prec="f64")
        st.close()
        return np.array([r.p for r in res])

    t = time.perf_counter()
    c = gi.calibrate_scale(A, target_clicks, lambda cv: float(marginals(cv).sum()), iters=40)
    calib_s = time.perf_counter() - t
    _, lam = gi.takagi_real_symmetric(A)
    lam = np.sort(lam)[::-1]
    nbar = np.sinh(np.arctanh(c * lam)) ** 2
    rng = np.random.default_rng([seed, 1])
    marks = [1, 10, 100, n_samples]
    uni = [rng.choice(n, k, replace=False) for _ in range(n_samples)]
    uni_d = np.array([gi.subgraph_density(A, u) for u in uni])
    uni_o = np.array([inside[u].sum() for u in uni])
    out = {"graph": f"G({n},{p}) + planted {clique}-clique, seed {seed}", "k": k, "scale_c": c,
           "calibration_seconds": calib_s, "target_mean_clicks": target_clicks,
           "encoding": {"lambda_1": float(lam[0]), "lambda_2": float(lam[1]), "c_lambda_1": float(c * lam[0]),
                        "mean_photons_total": float(nbar.sum()),
                        "mean_photons_top_mode_share": float(nbar[0] / nbar.sum())},
           "uniform": {"mean_density": float(uni_d.mean()),
                       "best_after": {str(x): float(uni_d[:x].max()) for x in marks},
                       "mean_in_clique": float(uni_o.mean()), "expected_in_clique": k * clique / n,
                       "p_all_in_clique": 1.0 / math.comb(n, k) * math.comb(clique, k)}}
    for eta in etas:
        cov = gi.graph_covariance(A, c, eta)
        pm = marginals(cov)
        with tg.Context(0) as cs:
            cs.set_option(tg.OPT_CHAIN_CLICKS, 20)
            samples, st = cs.gbs_sample(cov, k, seed + int(100 * eta), n_samples)
            raw, st2 = cs.gbs_sample(cov, -1, seed + 7, raw_chains)
        dens = np.array([gi.subgraph_density(A, np.nonzero(sm)[0]) for sm in samples])
        ov = samples[:, inside].sum(axis=1)
        hist = np.bincount(raw.sum(axis=1), minlength=21).tolist()
        raw_in = raw[:, inside].sum()
        out[f"eta={eta}"] = {"mean_clicks": float(pm.sum()), "samples": n_samples, "seconds": st["seconds"],
                             "samples_per_s": n_samples / st["seconds"],
                             "acceptance": st["chains_accepted"] / st["chains_started"],
                             "mean_density": float(dens.mean()),
                             "best_after": {str(x): float(dens[:x].max()) for x in marks},
                             "mean_in_clique": float(ov.mean()), "max_in_clique": int(ov.max()),
                             "fraction_of_clicks_in_clique": float(ov.mean() / k),
                             "samples_all_in_clique": int((ov == k).sum()),
                             "click_prob_in_clique": float(pm[inside].mean()),
                             "click_prob_outside": float(pm[~inside].mean()),
                             "raw_click_histogram": hist,
                             "raw_fraction_of_clicks_in_clique": float(raw_in / max(raw.sum(), 1)),
                             "raw_chains_capped": st2["chains_capped"], "raw_chains": st2["chains_started"]}
        print(f"dense subgraph eta={eta}: {n_samples} samples in {st['seconds']:.1f} s", file=sys.stderr,
              flush=True)
    return out


def sampler_bench(ctx, n_samples=1000, displaced=False, dd_terms=False):
    """The postselected sampling workload: m = 100, Haar U, r = 0.6, 12 clicks
    (displaced: the same state with mean 0.3 N(0, 1) per quadrature, seed 52;
    dd_terms: double-double chain terms, TOR_OPT_CHAIN_PREC)."""
    import numpy as np
    import gbs_inputs as gi
    import paper_1810_00900_amd as tg
    cov = gi.state_config2()
    mean = gi.random_mean(100, np.random.default_rng(52), 0.3) if displaced else None
    ctx.set_option(tg.OPT_CHAIN_PREC, tg.PREC_DD if dd_terms else tg.PREC_F64)
    try:
        samples, st = ctx.gbs_sample(cov, 12, 2, n_samples, mean=mean)
    finally:
        ctx.set_option(tg.OPT_CHAIN_PREC, tg.PREC_F64)
    assert (samples.sum(axis=1) == 12).all()
    extra = {}
    if dd_terms:
        # the same chains with binary64 terms: a coin that falls within the
        # binary64 error of P(click) sends its chain elsewhere; the two
        # ordered sample lists are aligned (difflib) to count such chains
        import difflib
        f64s, st64 = ctx.gbs_sample(cov, 12, 2, n_samples, mean=mean)
        a = [bytes(r) for r in samples]
        b = [bytes(r) for r in f64s]
        same = sum(m.size for m in difflib.SequenceMatcher(None, a, b, autojunk=False).get_matching_blocks())
        extra = {"samples_not_in_f64_run": n_samples - same, "chains_f64_run": st64["chains_started"]}
    return {"workload": "m=100, Haar U, r=0.6, postselected on 12 clicks, seed 2"
                        + (", displaced (mean 0.3 N(0,1), seed 52)" if displaced else ""),
            "samples": n_samples, "seconds": st["seconds"], "samples_per_s": n_samples / st["seconds"],
            "chains": st["chains_started"], "acceptance": st["chains_accepted"] / st["chains_started"],
            "subset_dets_per_s": st["subsets"] / st["seconds"],
            "precision": "dd terms and K_j words" if dd_terms else "f64 terms, dd sums", **extra}


def serving_bench(ctx, nq=10000, workers=2):
    """10^4 marginal-pattern queries (n ~ U{8..24}) on four 800-mode states,
    in three forms on the same GPU: the persistent request loop (one resident
    kernel claiming the queries' work units), the host-worker server (fused
    launches from host threads) and one query per launch.  Closed-loop
    saturation of each, then Poisson arrivals at 0.5x and 0.8x of the
    persistent loop's saturation rate for all three, then the persistent loop
    with sampling batches (config-2 chains) mixed into the query stream."""
    import numpy as np

    import gbs_inputs as gi
    import paper_1810_00900_amd as tg
    covs = [gi.state_m800(s) for s in (30, 31, 32, 33)]
    qs = gi.config3_queries(nq)
    sts = [ctx.state(c) for c in covs]
    rng = np.random.default_rng(35)

    def pct(lat):
        return {"p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3)}

    def arrivals(rate):
        return np.cumsum(rng.exponential(1.0 / rate, nq)) if rate else None

    def run_server(make, rate, chains=None):
        srv = make()
        arr = arrivals(rate)
        t0 = time.perf_counter()
        pending = collections.deque()  # (kind, ticket) in submission order
        res, cres = [], []

        def read_oldest():
            kind, t = pending.popleft()
            if kind == "p":
                res.append(srv.wait(t))
            else:
                cres.append(srv.wait_chains(t))

        def submit(fn, *a):
            while True:
                try:
                    return fn(*a)
                except tg.TorError as e:  # not admitted (ring or memory full): read a result, retry
                    if e.status != tg.TOR_EAGAIN or not pending:
                        raise
                    read_oldest()

        for k, (s, n, p) in enumerate(qs):
            if arr is not None:
                while time.perf_counter() - t0 < arr[k]:
                    pass
            pending.append(("p", submit(srv.submit, sts[s], p)))
            if chains and k % chains["every"] == 0:
                pending.append(("c", submit(srv.submit_chains, chains["state"], chains["n_post"], 2, chains["next"],
                                            chains["batch"])))
                chains["next"] += chains["batch"]
        while pending:
            read_oldest()
        T = time.perf_counter() - t0
        st = srv.stats()
        srv.stop()
        lat = np.array([x[1] for x in res])
        out = {"queries_per_s": nq / T}
        out.update(pct(lat))
        if "launches" in st:
            out["kernel_launches"] = st["launches"]
        else:
            out["batches"] = st["batches"]
            out["max_batch"] = st["max_batch_seen"]
        if cres:
            out["chain_batches"] = len(cres)
            out["chains"] = int(sum(len(c[1]) for c in cres))
            out["chains_accepted"] = int(sum(int((c[1] == 1).sum()) for c in cres))
            out.update({"chain_batch_" + k: v for k, v in pct(np.array([c[2] for c in cres])).items()})
        return out

    def persistent():
        return tg.PServer(ctx)

    def hostworkers():
        return tg.Server(ctx, workers=workers, prec="dd", tol=1e-10, max_batch=4096)

    def single(rate):
        arr = arrivals(rate)
        arr = arr if arr is not None else np.zeros(nq)
        t0 = time.perf_counter()
        lat = np.empty(nq)
        for k, (s, n, p) in enumerate(qs):
            if rate:
                while time.perf_counter() - t0 < arr[k]:
                    pass
            ctx.probability(covs[s], p, prec="dd", tol=1e-10)
            lat[k] = time.perf_counter() - t0 - arr[k]
        T = time.perf_counter() - t0
        out = {"queries_per_s": nq / T}
        out.update(pct(lat))
        return out

    res = {"workload": "10^4 queries, n ~ U{8..24}, marginal click sets, 4 states m=800 (seeds 30-33), "
                       "queries seed 34, dd terms, tol 1e-10; Poisson arrivals seed 35 at fractions of the "
                       "persistent loop's closed-loop rate"}
    def phase(name, fn, *a):
        t = time.perf_counter()
        print(f"[bench] serving: {name} ...", file=sys.stderr, flush=True)
        res[name] = fn(*a)
        print(f"[bench] serving: {name} done in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)

    phase("persistent_closed_loop", run_server, persistent, None)
    X = res["persistent_closed_loop"]["queries_per_s"]
    phase("served_closed_loop", run_server, hostworkers, None)
    phase("one_per_launch_closed_loop", single, None)
    for f in (0.5, 0.8):
        phase(f"persistent_poisson_{f}x", run_server, persistent, f * X)
        phase(f"served_poisson_{f}x", run_server, hostworkers, f * X)
        phase(f"one_per_launch_poisson_{f}x", single, f * X)
    res["poisson_rates_qps"] = {"0.5x": 0.5 * X, "0.8x": 0.8 * X}
    st2 = ctx.state(gi.state_config2())
    chains = {"state": st2, "n_post": 12, "batch": 256, "every": 100, "next": 0}
    phase("persistent_mixed_sampling_0.5x", run_server, persistent, 0.5 * X, chains)
    res["persistent_mixed_sampling_0.5x"]["sampling"] = ("a batch of 256 config-2 chains (m=100, r=0.6, "
                                                         "postselection on 12 clicks) every 100 queries")
    st2.close()
    for s in sts:
        s.close()
    res["subsets_total"] = float(sum(2.0 ** n for _, n, _ in qs))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=28)
    ap.add_argument("--prec", default="dd", choices=["dd", "f64"])
    ap.add_argument("--variant", default="zero-mean", choices=["zero-mean", "displaced", "qd"],
                    help="the same n-click Torontonian on a displaced state (random mean) or with quad-double "
                         "terms; for profiling those kernels (the headline is the zero-mean default)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip per-n, sampler and serving measurements")
    ap.add_argument("--copy-calibration", action="store_true", help="only run the 1 GiB copy used to scale counters")
    ap.add_argument("--only", default=None,
                    help="run one extra measurement by name (e.g. serving, sampler) and print its JSON")
    ap.add_argument("--invert-only", action="store_true",
                    help="only invert the 800-mode state (dd, qd) and time full patterns on it (for profiling)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.invert_only:
        import gbs_inputs as gi
        import paper_1810_00900_amd as tg
        ctx = tg.Context(0)
        print(json.dumps(full_pattern_inverse(ctx, gi.state_m800(50))), flush=True)
        ctx.close()
        return
    if args.only:
        import gbs_inputs as gi
        import paper_1810_00900_amd as tg
        fns = {"serving": serving_bench, "serving_full_patterns": serving_full_patterns, "sampler": sampler_bench,
               "dense_subgraph": dense_subgraph, "paper_worst_case": paper_worst_case}
        ctx = tg.Context(0)
        print(json.dumps({args.only: fns[args.only](ctx)}), flush=True)
        ctx.close()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the subset sum would shard by prefix bits with one 24-byte exchange per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import gbs_inputs as gi
    import paper_1810_00900_amd as tg

    n = args.n
    cov = gi.state_m800(50)
    pattern = gi.config5_pattern(n)
    ctx = tg.Context(0)
    ctx.set_option(tg.OPT_TIMING, 1)
    mean = gi.random_mean(800, np.random.default_rng(51), 0.3) if args.variant == "displaced" else None
    prec = "qd" if args.variant == "qd" else args.prec

    def call():
        if mean is not None:
            return ctx.probability_displaced(cov, mean, pattern, prec=prec, tol=1e-8)
        return ctx.probability(cov, pattern, prec=prec, tol=1e-8)

    for _ in range(args.warmup):
        r = call()
    ctx.reset_stats()
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = call()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = ctx.stats()
    ms_per_step = wall / args.steps * 1e3
    subsets = 2.0 ** n * args.steps
    value = subsets / wall

    J = ctx.tuning(args.prec, n) if prec != "qd" else min(n, 8)
    ntasks = 2 ** (n - J)
    wave_ms = st["wave_ms"] / max(st["wave_launches"], 1)
    if args.variant == "zero-mean":
        wave_flops = tree_flops(n, top=J) * ntasks
        kname = wave_kernel_name(args.prec, J)
        achieved = wave_flops / (wave_ms * 1e-3) / 1e12
    else:
        # no algorithmic model for these trees: the roofline uses the executed
        # FP64 flops of the committed PMC pass when its sources still match
        kname = wave_kernel_name(args.prec, J, 1) if args.variant == "displaced" else f"wave_kernel_qd<{J},0>"
        wave_flops = None
        ex = measured_fp64(kname, wave_ms) if n == 28 else None
        achieved = ex["achieved"] if ex else None
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "subset-dets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"dd": "f64-dd", "f64": "f64", "qd": "f64-qd"}[prec],
        "data": "synthetic (seeded Haar-random 800-mode GBS state)",
        "config": {"workload": f"large single Torontonian: m=800 modes (Haar U, r~U[0.3,0.9], seed 50), "
                               f"marginal click pattern with n={n} (2^{n} subsets)"
                               + (", displaced state (mean 0.3 N(0,1) per quadrature, seed 51)"
                                  if args.variant == "displaced" else ""),
                   "m": 800, "n": n, "precision": prec, "task_modes": J},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_PEAK_TFLOPS if achieved else None,
                     "basis": "algorithmic" if args.variant == "zero-mean" else "executed (PMC)",
                     "traffic": (measured_traffic(kname) if n == 28 else None),
                     "kernel": kname,
                     "kernel_ms": wave_ms,
                     "algorithmic_flops_per_launch": wave_flops,
                     "executed": (measured_fp64(kname, wave_ms) if n == 28 else None)},
        "phases_ms_per_step": {"expand": st["expand_ms"] / args.steps, "wave": st["wave_ms"] / args.steps,
                               "reduce": st["reduce_ms"] / args.steps},
        "result": {"p": r.p, "cancel_ratio": r.cancel_ratio, "rel_err_bound": r.rel_err_bound,
                   "prec_used": r.prec_used},
    }
    if args.variant != "zero-mean":
        out["metric"] = METRIC + f" ({args.variant} variant)"
    if args.variant == "zero-mean" and prec == "dd":
        # the metric covers n = 20..28: whole calls at n = 20 and 24 beside the
        # headline (frac over the call and over its kernels, algorithmic flops)
        pn = per_n_rates(ctx, cov, "dd", ns=(20, 24))
        out["roofline_per_n"] = {k: {"subset_dets_per_s": v["subset_dets_per_s"], "ms_per_call": v["ms"],
                                     "frac_call": v["frac_call"], "frac_kernels": v["frac_kernels"]}
                                 for k, v in pn.items()}
        out["roofline_per_n"]["20_batch64"] = batch_rate(ctx, cov, 20, 64)
        kms = (st["wave_ms"] + st["expand_ms"] + st["reduce_ms"]) / args.steps
        out["roofline_per_n"][str(n)] = {"subset_dets_per_s": value, "ms_per_call": ms_per_step,
                                         "frac_call": tree_flops(n) * args.steps / wall / 1e12 / FP64_PEAK_TFLOPS,
                                         "frac_kernels": tree_flops(n) / (kms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS}

    def step(name, fn, *a, **kw):  # one extra measurement, with a progress line on stderr
        t = time.perf_counter()
        out[name] = fn(*a, **kw)
        print(f"bench: {name} done in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)

    if not args.no_extras and args.variant == "zero-mean":
        mu = gi.random_mean(800, np.random.default_rng(51), 0.3)
        step("per_n", per_n_rates, ctx, cov, args.prec)
        step("per_n_f64_terms", per_n_rates, ctx, cov, "f64")
        step("per_n_full_pattern", per_n_rates, ctx, cov, args.prec, ns=(20, 28), full=True)
        step("per_n_qd_terms", per_n_rates, ctx, cov, "qd", ns=(20, 24, 28))
        step("per_n_full_pattern_qd", per_n_rates, ctx, cov, "qd", ns=(20, 28), full=True)
        step("full_pattern_inverse", full_pattern_inverse, ctx, cov)
        step("full_pattern_inverse_displaced", full_pattern_inverse, ctx, cov, mean=mu)
        step("per_n_displaced", per_n_rates, ctx, cov, args.prec, ns=(20, 24, 28), mean=mu)
        step("per_n_displaced_f64_terms", per_n_rates, ctx, cov, "f64", ns=(20, 24, 28), mean=mu)
        step("per_n_displaced_qd_terms", per_n_rates, ctx, cov, "qd", ns=(20, 24), mean=mu)
        step("per_n_full_pattern_displaced_qd", per_n_rates, ctx, cov, "qd", ns=(20,), full=True, mean=mu)
        step("sampler", sampler_bench, ctx)
        step("sampler_dd_terms", sampler_bench, ctx, dd_terms=True)
        step("sampler_displaced", sampler_bench, ctx, n_samples=200, displaced=True)
        step("paper_worst_case", paper_worst_case, ctx)
        step("paper_worst_case_qd", paper_worst_case, ctx, sizes=((16, 512), (18, 648), (20, 800)), prec="qd")
        step("dense_subgraph", dense_subgraph, ctx)
        step("serving", serving_bench, ctx)
        step("serving_full_patterns", serving_full_patterns, ctx)
    ctx.close()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(cov, pattern, n)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
