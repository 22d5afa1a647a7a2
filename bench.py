"""Benchmark of the particle-inference hot path on one MI355X.

Workload (one step = one ppl_importance call = the whole path): conjugate
Bayesian linear regression, d = 16 weights, D = 10^4 rows, N = 2^20 particles,
prior proposal, FP32 likelihood with FP64 log-sum-exp / ESS / posterior mean.
Inputs are synthetic (seeded, see synthetic/) and resident in HBM before the
timed region.  The metric is particle-likelihood evaluations per second
(N * D per step).

Printed as one JSON line, with
  roofline     -- the dominant kernel (blr_is_kernel) timed with HIP events on
                  its launch stream during the timed steps, against MI355X's
                  published FP32 vector peak (157.3 TFLOP/s, packed FP32), with
                  the fraction of the unpacked FMA issue ceiling the library can
                  reach (it is compiled without packed FP32) beside it as frac_attainable:
                  algorithmic work 34 FLOP per evaluation (16 FMA residual +
                  1 FMA square-accumulate);
  cpu_baseline -- the CPU oracle on a bounded sample of the same workload.

Other configurations print the same fields for their own workload:
  blr-stats         the same BLR workload with the likelihood from sufficient
                    statistics (X^T X, X^T y, y^T y once per call, then O(d^2)
                    FP64 per particle): particles per second, roofline of the
                    particle kernel's quadratic form against the FP64 peak
  poly, poly-paper  polynomial fit IS (FP64), 10^4 and 2 x 10^6 particles
  mcmc-poly         lightweight Metropolis-Hastings on the polynomial model (FP64):
                    2^16 chains x 1000 iterations over the C0 data, chain
                    iterations per second
  enum-hmm          exact inference by enumeration: every path of a 4-state
                    hidden Markov model over 20 steps (2^40 paths, FP64), paths
                    per second; roofline of the summing pass (two FMA per path)
                    against the FP64 vector peak
  lgssm             bootstrap SMC on the linear-Gaussian state space model
  gmm-batched       batched SMC over 256 mixture instances (autotuned first)
  resample-gather   resampling fused with the state gather, roofline against HBM
  proposal-poly/gmm ESS/s of the learned proposal at fixed log-evidence error
  proposal-train    simulated training pairs per second (MFMA rate with --no-graph)
  peaks             measured instruction and copy rates (not a hot-path line)

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu]
                       [--config blr|blr-stats|poly|poly-paper|mcmc-poly|enum-hmm|lgssm|gmm-batched|resample-gather|proposal-poly|
                                 proposal-gmm|proposal-train|peaks]
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X figures used as denominators.
CU, CLOCK_HZ, SIMD_PER_CU, LANES_PER_SIMD = 256, 2.4e9, 4, 16
FP32_VALU_UNPACKED_TFLOPS = CU * SIMD_PER_CU * LANES_PER_SIMD * 2 * CLOCK_HZ / 1e12   # 78.6
FP32_VALU_PUBLISHED_TFLOPS = 157.3        # needs packed FP32, which the library's compile flags disable
FP64_VALU_TFLOPS = 78.6

FLOP_PER_EVAL_BLR = 34                    # 17 FMA per (particle, row) at d = 16
# Committed PMC byte counts per configuration: (summary file under profiles/, the
# sources whose hash keys it).  A count is used only while the hash matches.
_CS = "paper_2010_08454_amd/csrc/"
TRAFFIC_FILES = {
    "blr": ("blr_is_kernel_traffic.txt", (_CS + "importance.hip", _CS + "blr.h", _CS + "device.h")),
    "blr-stats": ("blr_stats_is_kernel_traffic.txt", (_CS + "blr_stats.hip", _CS + "blr.h", _CS + "device.h")),
    "lgssm": ("smc_persistent_kernel_traffic_lgssm-N2p20-T1000.txt",
              (_CS + "smc.hip", _CS + "smc.h", _CS + "device.h")),
    "gmm-batched": ("smc_batched_kernel_traffic_gmm-batched-256inst-N2p16.txt",
                    (_CS + "batched.hip", _CS + "batched.h", _CS + "device.h")),
    "resample-gather": ("ancestor_gather_kernel_traffic.txt", (_CS + "resample.hip", _CS + "device.h")),
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="blr",
                    choices=["blr", "blr-stats", "poly", "poly-paper", "mcmc-poly", "enum-hmm", "lgssm", "gmm-batched",
                             "resample-gather",
                             "proposal-poly",
                             "proposal-gmm", "proposal-train", "peaks"])
    ap.add_argument("--pairs-log2", type=int, default=22, help="proposal-train: log2 of the simulated pairs")
    ap.add_argument("--no-graph", action="store_true", help="proposal-train: launch each step's kernels eagerly")
    ap.add_argument("--batch", type=int, default=0, help="proposal: training batch (default 4096)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--diagnose", action="store_true",
                    help="proposal-gmm: ESS/N of the learned proposal on held-out prior datasets and on the observed one")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle sample")
    ap.add_argument("--particles", type=int, default=0,
                    help="lgssm: particle count (default 2^20); resample-gather: (default 2^24)")
    ap.add_argument("--ess-frac", type=float, default=0.5, help="lgssm: resampling threshold")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy (reference for HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain device-to-device copy of known size: 256 MiB read + 256 MiB written
    per launch, the reference that scales the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = 64 << 20                                   # floats: 256 MiB
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n}), flush=True)


# Micro-benchmark kinds of libppl_peaks.so: (name, FLOP or ops per lane-instruction, unit, published peak)
PEAK_KINDS = [("fma_f32", 2, "TFLOP/s", 157.3), ("fma_f64", 2, "TFLOP/s", 78.6), ("exp_f32", 1, "Top/s", None),
              ("log_f32", 1, "Top/s", None), ("sin_f32", 1, "Top/s", None), ("mulhi_u32", 1, "Top/s", None),
              ("mfma_bf16", 16 * 16 * 32 * 2 // 64, "TFLOP/s", 2500.0)]


def bench_peaks(torch, dev, stream):
    """Measured rates of the instruction kinds the roofline fractions are priced
    against (libppl_peaks.so), beside MI355X's published figures: 2048
    workgroups of 256 lanes, eight independent chains per lane, each kernel
    sized to about 20 ms and timed with HIP events; and a 1 GiB device copy."""
    import ctypes
    L = ctypes.CDLL(os.path.join(ROOT, "paper_2010_08454_amd", "libppl_peaks.so"))
    L.peak_alu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    L.peak_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p]
    blocks = CU * 8
    out = torch.empty(blocks * 256, device=dev)
    sp = ctypes.c_void_p(stream.cuda_stream)

    def timed(fn, reps):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(reps):
            fn()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / reps

    res = {}
    for kind, (name, per, unit, pub) in enumerate(PEAK_KINDS):
        per_iter = L.peak_ops_per_iter(kind)

        def run(it):
            assert L.peak_alu(kind, blocks, it, ctypes.c_void_p(out.data_ptr()), sp) == 0
        iters = 64
        ms = timed(lambda: run(iters), 1)
        iters = max(64, int(iters * 20.0 / max(ms, 1e-3)))
        ms = timed(lambda: run(iters), 5)
        rate = blocks * 256 * iters * per_iter * per / (ms / 1e3) / 1e12
        res[name] = {"rate": round(rate, 2), "unit": unit, "published": pub, "ms": round(ms, 3), "iters": iters}
    n4 = (1 << 30) // 16
    src = torch.ones(n4 * 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for cb in (CU * 4, CU * 16):
        ms = timed(lambda: L.peak_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n4, cb, sp), 10)
        res[f"hbm_copy_{cb}wg"] = {"rate": round(2 * n4 * 16 / (ms / 1e3) / 1e9, 1), "unit": "GB/s", "published": 8000.0,
                                   "ms": round(ms, 4)}
    print(json.dumps({"metric": "measured peak rates", "n_gpus": 1, "data": "synthetic", "peaks": res,
                      "note": "fp32 FMA issue without packed FP32 (disabled in the library's compile flags) peaks at 78.64 TFLOP/s; "
                              "the published 157.3 assumes packed FP32"}), flush=True)


def cpu_model():
    """Host CPU model name (the `lscpu` "Model name" field, read from /proc/cpuinfo)."""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.lower().startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_rate(run, n_lo, n_hi, target_s, threads=None):
    """Time the oracle call run(n) on a particle count sized for about target_s
    seconds (a short calibration at n_lo, capped at n_hi; when even n_hi is
    shorter, the call is repeated).  threads: host threads for this measurement
    (None: the oracle's default).  Returns (n per second, n, repeats, seconds,
    threads used)."""
    import oracle
    oracle.build()
    prev = oracle.num_threads()
    if threads is not None:
        oracle.set_num_threads(threads)
    try:
        used = oracle.num_threads()
        t0 = time.perf_counter()
        run(n_lo)
        rate = n_lo / max(time.perf_counter() - t0, 1e-6)
        n = int(min(n_hi, max(n_lo, 2 ** round(math.log2(max(rate * target_s, 1.0))))))
        reps, dt = 0, 0.0
        while reps == 0 or (n == n_hi and dt < target_s * 0.6 and reps < 1000):
            t0 = time.perf_counter()
            run(n)
            dt += time.perf_counter() - t0
            reps += 1
    finally:
        oracle.set_num_threads(prev)
    return reps * n / dt, n, reps, dt, used


def cpu_record(run, n_lo, n_hi, per_n, unit, what, target_s):
    """cpu_baseline object: the oracle with all its threads (about target_s
    seconds) and with one thread (about a third of that), host CPU model."""
    r_all, n, reps, dt, used = oracle_rate(run, n_lo, n_hi, target_s)
    r_one, n1, reps1, dt1, _ = oracle_rate(run, n_lo, n_hi, target_s / 3, threads=1)
    return {"value": r_all * per_n, "unit": unit, "cores": used, "kind": "oracle",
            "value_1_thread": r_one * per_n, "cpu_model": cpu_model(),
            "usable_cores": len(os.sched_getaffinity(0)),
            "sample": f"{what(n)}, {reps} run(s), {dt:.1f} s on {used} threads; 1 thread: {what(n1)}, "
                      f"{reps1} run(s), {dt1:.1f} s; FP64 oracle"}


def cpu_baseline_blr(X, y, n_full, seed, target_s=15.0):
    """The oracle's BLR importance sampling on a particle sample of the same workload."""
    import oracle
    run = lambda n: oracle.importance(oracle.MODEL_BLR, X, y, n, seed, dim=X.shape[1])
    what = lambda n: ("the full workload" if n == n_full else f"{n} of the {n_full} particles") + f" over all {y.size} rows"
    return cpu_record(run, 1 << 12, n_full, y.size, "particle-likelihood evals/s", what, target_s)


def cpu_baseline_mcmc(x, y, C, T, burn, seed, target_s=15.0):
    """The oracle's chains (all T iterations each) on a sample of the chains."""
    import oracle
    run = lambda k: oracle.mcmc_poly(x, y, k, T, seed, burn_in=burn)
    what = lambda k: f"{k} of the {C} chains, {T} iterations each"
    return cpu_record(run, 64, C, T, "chain-iterations/s", what, target_s)


def cpu_baseline_lgssm(y, seed, target_s=15.0):
    """The oracle's SMC on a particle sample sized for about `target_s` seconds."""
    import oracle
    y64 = y.astype("float64")
    run = lambda n: oracle.smc(oracle.MODEL_LGSSM, y64, n, seed)
    what = lambda n: f"{n} of the 2^20 particles over all {y.size} steps"
    return cpu_record(run, 1 << 12, 1 << 20, y.size, "particle-step evals/s", what, target_s)


def code_hash(sources):
    """SHA-256 of the sources with their comments removed: counter summaries
    stay valid across comment edits and go stale on any change to the code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for src in sources:
        text = open(os.path.join(ROOT, src)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update("\n".join(ln.rstrip() for ln in text.splitlines() if ln.strip()).encode())
    return h.hexdigest()


def measured_traffic(config):
    """HBM bytes per launch from the committed rocprofv3 PMC summary of the
    configuration's dominant kernel, or None when there is none or the kernel's
    sources changed since the counters were taken."""
    import hashlib
    if config not in TRAFFIC_FILES:
        return None
    fname, sources = TRAFFIC_FILES[config]
    path = os.path.join(ROOT, "profiles", fname)
    if not os.path.exists(path):
        return None
    kv = {}
    for ln in open(path):
        if ":" in ln and not ln.startswith("#"):
            k, v = ln.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != code_hash(sources):
        return None
    try:
        return int(float(kv["fetch_bytes_per_launch"]) + float(kv["write_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


def cpu_baseline_poly(x, y, n, seed, target_s=15.0):
    import oracle
    run = lambda k: oracle.importance(oracle.MODEL_POLY, x, y, k, seed)
    what = lambda k: f"{k} particles over all {y.size} points"
    return cpu_record(run, min(n, 1 << 12), n, y.size, "particle-likelihood evals/s", what, target_s)


HBM_GBS = 8000.0
GATHER_FIELDS = 16


def cpu_baseline_enum(y, pi0, A, mu, sigma, target_s=15.0):
    """The oracle's enumeration on the first T' steps of the same model, T' the
    largest length it finishes in about target_s seconds.  Its cost per path
    grows linearly with the length, so the rate is scaled by T' / T to paths of
    the full length."""
    import oracle
    oracle.build()
    K, T = len(pi0), len(y)
    hyper = oracle.hmm_hyper(pi0, A, mu, sigma)

    def measure(budget, threads):
        prev = oracle.num_threads()
        if threads is not None:
            oracle.set_num_threads(threads)
        try:
            used = oracle.num_threads()
            Tp = min(T, max(2, int(math.log(2e5) / math.log(K))))
            t0 = time.perf_counter()
            oracle.enumerate_hmm(y[:Tp], hyper)
            per_path = (time.perf_counter() - t0) / K ** Tp
            while Tp < T and per_path * K ** (Tp + 1) <= budget:
                Tp += 1
            t0 = time.perf_counter()
            oracle.enumerate_hmm(y[:Tp], hyper)
            dt = time.perf_counter() - t0
            return K ** Tp / dt * Tp / T, Tp, dt, used
        finally:
            oracle.set_num_threads(prev)

    v, Tp, dt, used = measure(target_s, None)
    v1, Tp1, dt1, _ = measure(target_s / 3, 1)
    return {"value": v, "unit": "paths/s", "cores": used, "kind": "oracle", "value_1_thread": v1,
            "cpu_model": cpu_model(), "usable_cores": len(os.sched_getaffinity(0)),
            "sample": f"all {K}^{Tp} paths of the first {Tp} steps ({dt:.1f} s, {used} threads); 1 thread: "
                      f"{K}^{Tp1} paths of {Tp1} steps ({dt1:.1f} s); rates scaled by T'/{T} to {T}-step paths; "
                      "FP64 oracle"}


def bench_enum(args, ppl, synthetic, torch, dev, stream):
    """Exact inference by enumeration over a hidden Markov model: K = 4 states,
    T = 20 steps, 2^40 paths (synthetic chain and observations, see
    synthetic.hmm_instance).  One step = one ppl_enumerate call (emission
    table, the maximum pass, the summing pass, merges).  Roofline: the summing
    pass at 2 + 1/K FLOP per path (an FMA of the path's weight into its last
    site's sum, and one product per K sibling paths for their parent's
    subtotal) against the FP64 vector peak.  The maximum pass is reported
    beside it at 3/K operations per path: per K sibling paths the add of their
    parent's weight, the add of the last site's row maximum and a max."""
    K, T = 4, 20
    pi0, A, mu, sigma, y, _ = synthetic.hmm_instance(K, T)
    dy = torch.from_numpy(y).to(dev)
    data = ppl.hmm_data(dy, pi0, A, mu, sigma)
    ws = ppl.workspace(ppl.ppl_workspace_size(ppl.PPL_MODEL_HMM, data, 1, ppl.PPL_ALGO_ENUM), dev)
    scal = torch.empty(4, dtype=torch.float64, device=dev)
    marg = torch.empty((T, K), dtype=torch.float64, device=dev)
    mp = torch.empty(T, dtype=torch.int32, device=dev)

    def step():
        ppl.ppl_enumerate(ppl.PPL_MODEL_HMM, data, ws=ws, stream=stream, scalars=scal, marginals=marg, map_path=mp)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ppl.ppl_timing_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    s_ms, s_n = ppl.ppl_timing_query("enum_sum_kernel")
    m_ms, m_n = ppl.ppl_timing_query("enum_max_kernel")
    ppl.ppl_timing_enable(False)
    sc = scal.cpu().numpy()
    assert sc[3] == 0 and math.isfinite(sc[0]), f"device status {sc[3]}"
    paths = float(K) ** T
    ms_per_step = total_ms / args.steps
    s_avg, m_avg = s_ms / max(s_n, 1), m_ms / max(m_n, 1)
    flop_per_launch = (2 + 1 / K) * paths
    achieved = flop_per_launch / (s_avg / 1e3) / 1e12
    out = {"metric": "paths/s", "value": paths / (ms_per_step / 1e3), "unit": "paths/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
           "data": "synthetic (seeded generators, inputs resident in HBM)",
           "config": {"workload": "enum-hmm", "model": "hidden Markov model, Gaussian emissions",
                      "states": K, "steps": T, "paths": paths, "precision": "fp64"},
           "log_evidence": float(sc[0]), "map_log_joint": float(sc[2]),
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                        "frac": round(achieved / FP64_VALU_TFLOPS, 4), "traffic": None,
                        "kernel": "enum_sum_kernel", "kernel_ms": round(s_avg, 4), "kernel_launches": s_n,
                        "flop_per_launch": flop_per_launch,
                        "max_pass": {"kernel": "enum_max_kernel", "kernel_ms": round(m_avg, 4),
                                     "ops_per_path": round(3 / K, 4),
                                     "achieved_top_s": round(3 / K * paths / (m_avg / 1e3) / 1e12, 3),
                                     "peak_top_s": round(FP64_VALU_TFLOPS / 2, 2)}}}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_enum(y, pi0, A, mu, sigma, target_s=args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_resample_gather(args, ppl, synthetic, torch, dev, stream):
    """Systematic resampling fused with the gather of the particle state, at the
    state size of the batched mixture workload: N = 2^24 particles x 16 FP32
    fields (1.07 GB, the bytes of 256 instances x 2^16 particles x 2K = 16
    fields), FP32 log-weights ~ N(0, 1).  One step = one ppl_resample_gather
    call (quantisation, tile scans, tile prefix, fused ancestor search and
    gather).  Roofline: ancestor_gather_kernel against HBM, algorithmic bytes
    per particle 2 x 16 x 4 (state read + write) + 8 (its prefix-sum entry)."""
    N, F, seed = args.particles or (1 << 24), GATHER_FIELDS, 1
    lw_h = synthetic.logweights(N, "normal", seed=3, scale=1.0)
    lw = torch.from_numpy(lw_h).to(dev)
    gen = torch.Generator(device=dev)
    gen.manual_seed(7)
    state = torch.randn((F, N), generator=gen, device=dev, dtype=torch.float32)
    out = torch.empty_like(state)
    ws = ppl.workspace(ppl.ppl_workspace_size(0, None, N, ppl.PPL_ALGO_RESAMPLE), dev)

    def step(k):
        ppl.ppl_resample_gather(lw, state, seed, step=k, out=out, ws=ws, stream=stream)

    for k in range(args.warmup):
        step(k)
    torch.cuda.synchronize()
    ppl.ppl_timing_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for k in range(args.steps):
        step(args.warmup + k)
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    k_ms, k_n = ppl.ppl_timing_query("ancestor_gather_kernel")
    ppl.ppl_timing_enable(False)
    ms = total_ms / args.steps
    k_avg = k_ms / max(k_n, 1)
    bytes_per_launch = N * (2 * F * 4 + 8)
    achieved = bytes_per_launch / (k_avg / 1e3) / 1e9
    # whole call: log-weights read twice (tile maxima, quantised scan), prefix sums written once
    call_bytes = N * (4 + 4 + 8) + bytes_per_launch
    workload = {"workload": "resample-gather", "particles": N, "state_fields": F, "state_dtype": "f32",
                "state_bytes": F * N * 4, "log_weights": "fp32 ~ N(0, 1)",
                "call_gb_per_s": round(call_bytes / (ms / 1e3) / 1e9, 1)}
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_GBS, 4),
                "traffic": measured_traffic("resample-gather"),
                "kernel": "ancestor_gather_kernel", "kernel_ms": round(k_avg, 4), "kernel_launches": k_n,
                "bytes_per_launch": bytes_per_launch}
    res = {"metric": "resampled particles/s", "value": N / (ms / 1e3), "unit": "particles/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic (seeded generators, inputs resident in HBM)", "config": workload,
           "roofline": roofline}
    if not args.no_cpu:
        res["cpu_baseline"] = cpu_baseline_resample(lw_h, state.cpu().numpy(), seed)
    print(json.dumps(res), flush=True)


def cpu_baseline_resample(lw, state, seed, target_s=10.0):
    """The oracle's resampling plus the gather by index on a particle sample
    sized for about `target_s` seconds."""
    import numpy as np
    import oracle
    oracle.build()
    n = min(lw.size, 1 << 18)
    t0 = time.perf_counter()
    a, _ = oracle.resample(lw[:n].astype(np.float64), seed)
    np.ascontiguousarray(state[:, :n][:, a])
    dt = time.perf_counter() - t0
    n = int(min(lw.size, max(n, 2 ** round(math.log2(n * target_s / max(dt, 1e-6))))))
    lw64 = lw[:n].astype(np.float64)
    sub = np.ascontiguousarray(state[:, :n])
    reps, dt = 0, 0.0
    while reps == 0 or (dt < target_s * 0.6 and reps < 20):
        t0 = time.perf_counter()
        a, _ = oracle.resample(lw64, seed)
        np.ascontiguousarray(sub[:, a])
        dt += time.perf_counter() - t0
        reps += 1
    what = "the full workload" if n == lw.size else f"{n} of the {lw.size} particles"
    return {"value": reps * n / dt, "unit": "particles/s", "cores": 1, "kind": "oracle",
            "value_1_thread": reps * n / dt, "cpu_model": cpu_model(), "usable_cores": len(os.sched_getaffinity(0)),
            "sample": f"{what} ({state.shape[0]} fields), {reps} run(s): oracle resampling + gather by index "
                      f"({dt:.1f} s; the resampling scan is sequential, so one thread)"}


BF16_MFMA_TFLOPS = 2500.0
GEMM_FLOP_PER_PAIR = 2 * 425984      # forward 3 layers + 2 input-gradient + 3 weight-gradient products
# the kernels that run the network's products: the fused pass (forward, loss
# head, input gradients) and the grouped weight-gradient launch, or the
# per-product GEMMs when PPL_TRAIN_UNFUSED=1
PRODUCT_KERNELS = ("fused_pass_kernel", "wgrad_group_kernel", "gemm_nt_kernel")
SEEDS_PER_RUNG = 16
RMSE_TARGET = 0.05


def lse_merge(parts):
    """log-sum-exp merge of FP64 partials (max, s1, s2) over disjoint particle sets."""
    m = max(p[0] for p in parts)
    s1 = sum(p[1] * math.exp(p[0] - m) for p in parts)
    s2 = sum(p[2] * math.exp(2 * (p[0] - m)) for p in parts)
    return m, s1, s2


def poly_log_evidence(x, y, sd=10.0, degrees=(2, 3, 4, 5)):
    """Exact log-evidence of the polynomial model (factor -1/2 sum of squared
    residuals, no 2 pi constant; n uniform on `degrees`, c ~ N(0, sd^2 I)).
    Given n the factor is Gaussian in c, so with Phi the D x n design matrix,
    G = Phi^T Phi, b = Phi^T y and A = I / sd^2 + G:
      log Z_n = -1/2 log det(I + sd^2 G) - 1/2 (y^T y - b^T A^{-1} b),
    and log Z = log mean_n Z_n."""
    import numpy as np
    x, y = np.asarray(x, np.float64), np.asarray(y, np.float64)
    lz = []
    for n in degrees:
        Phi = np.vander(x, n, increasing=True)
        G, b = Phi.T @ Phi, Phi.T @ y
        logdet = np.linalg.slogdet(np.eye(n) + sd * sd * G)[1]
        lz.append(-0.5 * logdet - 0.5 * (y @ y - b @ np.linalg.solve(np.eye(n) / (sd * sd) + G, b)))
    lz = np.array(lz) - math.log(len(degrees))
    m = lz.max()
    return float(m + math.log(np.exp(lz - m).sum()))


def bench_proposal(args, ppl, synthetic, torch, dev, stream):
    """Learned proposal against the prior proposal: ESS per second of the
    inference call at the smallest power-of-two particle count whose log Z-hat
    RMSE over 16 seeds is within 0.05 of the reference.  The reference is the
    exact log-evidence for the polynomial model (conjugate Gaussian given the
    degree, summed over the four degrees) and the prior proposal's FP64
    estimate at 2^34 particles for the mixture, which has no closed form."""
    poly = args.config == "proposal-poly"
    if poly:
        x, y = synthetic.poly_data(D=1000, seed=synthetic.SEED_POLY_LEARN)
        data = ppl.make_data(torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev))
        model, D, K, ref_chunks = ppl.PPL_MODEL_POLY, 1000, 0, 4
        kname, op_per_eval = "poly_mix_is_kernel", 10
        workload = {"workload": "learned-proposal-poly", "model": "polynomial fit (degree ~ U{2..5})", "points": D}
    else:
        y = synthetic.gmm_learn_data(K=5, D=100)
        data = ppl.make_data(None, torch.from_numpy(y).to(dev), dim=5)
        model, D, K, ref_chunks = ppl.PPL_MODEL_GMM, 100, 5, 16
        # FP32 issue slots per (particle, datum), transcendentals at two (their measured half rate):
        # per component 2 FMA (shifted square), max, exponent scale, v_exp (2), accumulate = 7;
        # per datum v_log (2) + scale + accumulate into the log-weight = 4
        kname, op_per_eval = "gmm_mix_is_kernel", 7 * 5 + 4
        workload = {"workload": "learned-proposal-gmm", "model": "Gaussian mixture, K = 5", "points": D}
    sc = torch.empty(8, dtype=torch.float64, device=dev)
    if poly:
        ref = poly_log_evidence(x, y)
        ref_info = {"log_evidence": round(ref, 6), "kind": "exact (conjugate per degree, summed over degrees)"}
    else:
        chunk = 1 << 30
        ws = ppl.workspace(ppl.ppl_workspace_size(model, data, chunk, ppl.PPL_ALGO_IS), dev)
        parts = []
        for c in range(ref_chunks):
            ppl.ppl_importance(model, data, chunk, 10_000 + c, ws=ws, stream=stream, scalars=sc)
            parts.append(tuple(sc.cpu().numpy()[4:7]))
        m, s1, s2 = lse_merge(parts)
        ref = m + math.log(s1) - math.log(chunk * ref_chunks)
        ref_ess = s1 * s1 / s2
        # the estimate's own standard error: sqrt(1 / ESS - 1 / n) in log Z (delta method)
        ref_info = {"log_evidence": round(ref, 5), "ess": round(ref_ess, 1), "particles": chunk * ref_chunks,
                    "proposal": "prior, fp64", "std_error": round(math.sqrt(max(1 / ref_ess - 1 / (chunk * ref_chunks), 0)), 4)}
        del ws

    # training defaults per model (a sweep of batch, learning rate and decay at 2^22 pairs)
    B = args.batch or (512 if poly else 256)
    lr, decay = (1e-3, False) if poly else (3e-3, True)
    pairs = 1 << 22
    cfg = ppl.train_config(pairs, B, D, dim=K, lr=lr, use_graph=True, lr_decay_steps=pairs // B if decay else 0,
                           lr_final_frac=0.02)
    wts = ppl.ppl_proposal_init(1, stream=stream)
    tws = ppl.workspace(ppl.ppl_proposal_train_workspace_size(model, cfg), dev)
    trace = torch.empty(pairs // B, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ppl.ppl_proposal_train(model, cfg, 1, wts, loss_trace=trace, ws=tws, stream=stream)
    torch.cuda.synchronize()
    train_ms = (time.perf_counter() - t0) * 1e3
    tr = trace.cpu().numpy()
    # MFMA rate of the network products: a few eager steps on a copy with kernel timing on
    probe_steps = 16
    wcopy = wts.clone()
    pcfg = ppl.train_config(probe_steps * B, B, D, dim=K, lr=lr)
    ppl.ppl_timing_enable(True)
    ppl.ppl_proposal_train(model, pcfg, 1, wcopy, ws=tws, stream=stream)
    torch.cuda.synchronize()
    g_ms = sum(ppl.ppl_timing_query(k)[0] for k in PRODUCT_KERNELS)
    ppl.ppl_timing_enable(False)
    gemm_tflops = GEMM_FLOP_PER_PAIR * B * probe_steps / (g_ms / 1e3) / 1e12
    # adaptive tempering of the proposal for this dataset (pilot ESS, no reference)
    t0 = time.perf_counter()
    widen, pilot = ppl.ppl_proposal_pick_widen(model, data, wts, stream=stream)
    pilot_ms = (time.perf_counter() - t0) * 1e3

    def ladder(learned, n_lo, n_hi):
        iws = None
        for lg in range(n_lo, n_hi + 1):
            N = 1 << lg
            need = (ppl.ppl_proposal_infer_workspace_size(model, data, N) if learned
                    else ppl.ppl_workspace_size(model, data, N, ppl.PPL_ALGO_IS))
            iws = ppl.workspace(need, dev)
            est, ess, ms = [], [], []
            for sd in range(SEEDS_PER_RUNG):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                if learned:
                    ppl.ppl_proposal_infer(model, data, wts, N, 100 + sd, ws=iws, stream=stream, scalars=sc,
                                           widen=widen)
                else:
                    ppl.ppl_importance(model, data, N, 100 + sd, ws=iws, stream=stream, scalars=sc)
                e1.record(stream)
                torch.cuda.synchronize()
                v = sc.cpu().numpy()
                est.append(v[0])
                ess.append(v[1])
                ms.append(e0.elapsed_time(e1))
            rmse = math.sqrt(sum((e - ref) ** 2 for e in est) / len(est))
            if rmse <= RMSE_TARGET or lg == n_hi:
                mean_ess, mean_ms = sum(ess) / len(ess), sum(ms) / len(ms)
                return {"particles": N, "rmse": round(rmse, 4), "met": rmse <= RMSE_TARGET,
                        "ess": round(mean_ess, 2), "ms_per_call": round(mean_ms, 4),
                        "ess_per_s": mean_ess / (mean_ms / 1e3)}
        return None

    if args.diagnose and not poly:
        # held-out datasets drawn from the prior by the observed dataset's recipe (other seeds): if the
        # proposal is as poor there as on the observed dataset, the gap is the network's (capacity or
        # parameterisation), not a mismatch between the observed data and the training distribution
        Nd = 1 << 16
        dws = ppl.workspace(ppl.ppl_proposal_infer_workspace_size(model, data, Nd), dev)
        pws = ppl.workspace(ppl.ppl_workspace_size(model, data, Nd, ppl.PPL_ALGO_IS), dev)

        def ess_frac(d, learned_q, w=1.0, sd=500):
            if learned_q:
                ppl.ppl_proposal_infer(model, d, wts, Nd, sd, ws=dws, stream=stream, scalars=sc, widen=w)
            else:
                ppl.ppl_importance(model, d, Nd, sd, ws=pws, stream=stream, scalars=sc)
            return float(sc.cpu().numpy()[1]) / Nd

        held, held_prior = [], []
        for i in range(32):
            yi = synthetic.gmm_learn_data(K=5, D=100, seed=synthetic.SEED_GMM_LEARN + 7919 * (i + 1))
            di = ppl.make_data(None, torch.from_numpy(yi).to(dev), dim=5)
            held.append(ess_frac(di, True, sd=500 + i))
            held_prior.append(ess_frac(di, False, sd=500 + i))
        q = lambda v, f: float(sorted(v)[int(f * (len(v) - 1))])
        workload["diagnosis"] = {
            "particles": Nd,
            "held_out_learned_ess_over_n": {"min": q(held, 0), "median": q(held, 0.5), "max": q(held, 1)},
            "held_out_prior_ess_over_n": {"min": q(held_prior, 0), "median": q(held_prior, 0.5),
                                          "max": q(held_prior, 1)},
            "observed_learned_ess_over_n": ess_frac(data, True),
            "observed_learned_widened_ess_over_n": ess_frac(data, True, w=widen),
            "observed_prior_ess_over_n": ess_frac(data, False)}
        del dws, pws

    learned = ladder(True, 10, 24)
    prior = ladder(False, 10, 30)
    # kernel rate of the learned inference at its particle count
    N = learned["particles"]
    iws = ppl.workspace(ppl.ppl_proposal_infer_workspace_size(model, data, N), dev)
    ppl.ppl_timing_enable(True)
    for sd in range(args.steps):
        ppl.ppl_proposal_infer(model, data, wts, N, 100 + sd, ws=iws, stream=stream, scalars=sc, widen=widen)
    torch.cuda.synchronize()
    k_ms, k_n = ppl.ppl_timing_query(kname)
    ppl.ppl_timing_enable(False)
    k_avg = k_ms / max(k_n, 1)
    achieved = op_per_eval * N * D / (k_avg / 1e3) / 1e12
    # POLY: FP64 FLOP against the FP64 VALU peak; GMM: FP32 issue slots against the issue rate
    peak, unit = (FP64_VALU_TFLOPS, "TFLOP/s") if poly else (FP32_VALU_UNPACKED_TFLOPS / 2, "TOP/s")
    workload.update({"reference": ref_info,
                     "training": {"pairs": pairs, "batch": B, "steps": pairs // B, "ms": round(train_ms, 2),
                                  "loss_first": round(float(tr[:8].mean()), 4),
                                  "loss_last": round(float(tr[-8:].mean()), 4),
                                  "gemm_tflops": round(gemm_tflops, 2), "gemm_peak_tflops": BF16_MFMA_TFLOPS,
                                  "gemm_frac": round(gemm_tflops / BF16_MFMA_TFLOPS, 4), "lr": lr,
                                  "cosine_decay": decay},
                     "widen": {"chosen": widen, "pilot_ess": [round(e, 1) for e in pilot],
                               "candidates": list(ppl.WIDEN_CANDIDATES), "pilot_particles": 1 << 14,
                               "ms": round(pilot_ms, 2)},
                     "learned": learned, "prior": prior, "rmse_target": RMSE_TARGET,
                     "seeds_per_rung": SEEDS_PER_RUNG})
    out = {"metric": "ESS/s at log Z RMSE <= 0.05 (learned proposal)", "value": learned["ess_per_s"],
           "unit": "ESS/s", "n_gpus": 1, "steps": args.steps, "warmup": 0,
           "ms_per_step": learned["ms_per_call"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f64" if poly else "f32",
           "data": "synthetic (seeded generators, inputs resident in HBM)", "config": workload,
           "speedup_vs_prior": round(learned["ess_per_s"] / prior["ess_per_s"], 2) if prior else None,
           # when the prior proposal misses the target at every rung up to its largest particle count, the
           # ratio above compares against that largest rung, so it is a lower bound on the gain
           "speedup_is_lower_bound": bool(prior) and not prior["met"],
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 2), "unit": unit,
                        "frac": round(achieved / peak, 4), "traffic": None, "kernel": kname,
                        "kernel_ms": round(k_avg, 4), "kernel_launches": k_n,
                        "flop_per_launch": op_per_eval * N * D}}
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline_prior_ess(poly, x if poly else None, y, D, target_s=args.cpu_seconds)
    print(json.dumps(out), flush=True)


def bench_proposal_train(args, ppl, torch, dev, stream):
    """Training of the POLY proposal network alone (the network products are the
    MFMA work): simulated pairs per second, and the GEMM kernels' FLOP rate
    against the BF16 dense MFMA peak."""
    B = args.batch or 512
    pairs = 1 << args.pairs_log2
    steps = pairs // B
    cfg = ppl.train_config(pairs, B, 1000, lr=1e-3, use_graph=not args.no_graph)
    wts = ppl.ppl_proposal_init(1, stream=stream)
    tws = ppl.workspace(ppl.ppl_proposal_train_workspace_size(ppl.PPL_MODEL_POLY, cfg), dev)
    trace = torch.empty(steps, dtype=torch.float64, device=dev)
    warm = ppl.train_config(8 * B, B, 1000, lr=1e-3)
    ppl.ppl_proposal_train(ppl.PPL_MODEL_POLY, warm, 1, ppl.ppl_proposal_init(2, stream=stream), ws=tws, stream=stream)
    torch.cuda.synchronize()
    ppl.ppl_timing_enable(args.no_graph)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    ppl.ppl_proposal_train(ppl.PPL_MODEL_POLY, cfg, 1, wts, loss_trace=trace, ws=tws, stream=stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    out = {"metric": "simulated training pairs/s", "value": pairs / (ms / 1e3), "unit": "pairs/s", "n_gpus": 1,
           "steps": steps, "warmup": 8, "ms_per_step": round(ms / steps, 4), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic (pairs simulated from the model prior on the device)",
           "config": {"workload": "learned-proposal-training-poly", "pairs": pairs, "batch": B,
                      "graph": not args.no_graph, "loss_last": float(trace[-8:].mean())}}
    if args.no_graph:
        names = PRODUCT_KERNELS
        q = {k: ppl.ppl_timing_query(k) for k in names}
        g_ms = sum(v[0] for v in q.values())
        used = [k for k in names if q[k][1] > 0]
        achieved = GEMM_FLOP_PER_PAIR * pairs / (g_ms / 1e3) / 1e12
        out["roofline"] = {"bound": "mfma", "achieved": round(achieved, 3), "peak": BF16_MFMA_TFLOPS,
                           "unit": "TFLOP/s", "frac": round(achieved / BF16_MFMA_TFLOPS, 5), "traffic": None,
                           "kernel": "+".join(used), "kernel_ms_per_step": round(g_ms / steps, 5),
                           "kernel_launches": {k: q[k][1] for k in used}, "flop_per_pair": GEMM_FLOP_PER_PAIR}
    ppl.ppl_timing_enable(False)
    print(json.dumps(out), flush=True)


def cpu_baseline_prior_ess(poly, x, y, D, target_s=15.0):
    """The oracle's prior-proposal importance sampling on the same data: ESS per
    second on a particle count sized to about target_s seconds, with all the
    oracle's threads and with one."""
    import numpy as np
    import oracle
    from oracle import proposal as opr
    oracle.build()
    if poly:
        run = lambda k: float(oracle.importance(oracle.MODEL_POLY, x, y, k, 7)["ess"])
    else:
        yd = np.asarray(y, dtype=np.float64)

        def run(k):
            r = opr.gmm_prior_lw(7, 5, yd, np.arange(k))
            w = np.exp(r - r.max())
            return float(w.sum() ** 2 / (w * w).sum())

    def measure(budget, threads):
        prev = oracle.num_threads()
        if threads is not None:
            oracle.set_num_threads(threads)
        try:
            used = oracle.num_threads()
            n = 1 << 12
            t0 = time.perf_counter()
            run(n)
            dt = time.perf_counter() - t0
            n = max(n, int(n * budget / max(dt, 1e-3)))
            t0 = time.perf_counter()
            ess = run(n)
            return ess / (time.perf_counter() - t0), n, time.perf_counter() - t0, used
        finally:
            oracle.set_num_threads(prev)

    v, n, dt, used = measure(target_s, None)
    v1, n1, dt1, _ = measure(target_s / 3, 1)
    return {"value": v, "unit": "ESS/s", "cores": used, "kind": "oracle", "value_1_thread": v1,
            "cpu_model": cpu_model(), "usable_cores": len(os.sched_getaffinity(0)),
            "sample": f"prior-proposal importance sampling, one seed: {n} particles ({dt:.1f} s, {used} threads); "
                      f"{n1} particles ({dt1:.1f} s, 1 thread)"}


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(json.dumps({"error": "the library runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        copy_calibration()
        return
    import torch

    import synthetic
    import paper_2010_08454_amd as ppl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()
    if args.config == "proposal-train":
        bench_proposal_train(args, ppl, torch, dev, stream)
        return
    if args.config.startswith("proposal"):
        bench_proposal(args, ppl, synthetic, torch, dev, stream)
        return
    if args.config == "peaks":
        bench_peaks(torch, dev, stream)
        return
    if args.config == "resample-gather":
        bench_resample_gather(args, ppl, synthetic, torch, dev, stream)
        return
    if args.config == "enum-hmm":
        bench_enum(args, ppl, synthetic, torch, dev, stream)
        return

    if args.config == "blr":
        d, D, N, seed = 16, 10_000, 1 << 20, 1
        X, y, _ = synthetic.blr_data(D=D, d=d)
        dX, dy = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
        data = ppl.make_data(dX, dy, dim=d)
        model, kname = ppl.PPL_MODEL_BLR, "blr_is_kernel"
        nsum = d
        workload = {"workload": "blr-importance-sampling", "model": "conjugate Bayesian linear regression",
                    "d": d, "rows": D, "particles": N, "proposal": "prior",
                    "precision": "fp32 likelihood, fp64 normaliser"}
        flop_per_launch = FLOP_PER_EVAL_BLR * N * D
        peak, bound, unit, dtype = FP32_VALU_PUBLISHED_TFLOPS, "alu", "TFLOP/s", "f32"
    elif args.config == "blr-stats":
        d, D, N, seed = 16, 10_000, args.particles or (1 << 20), 1
        X, y, _ = synthetic.blr_data(D=D, d=d)
        dX, dy = torch.from_numpy(X).to(dev), torch.from_numpy(y).to(dev)
        data = ppl.make_data(dX, dy, dim=d)
        model, kname = ppl.PPL_MODEL_BLR_STATS, "blr_stats_is_kernel"
        nsum = d
        workload = {"workload": "blr-stats-importance-sampling",
                    "model": "conjugate Bayesian linear regression, likelihood from sufficient statistics",
                    "d": d, "rows": D, "particles": N, "proposal": "prior",
                    "precision": "fp32 latents, fp64 statistics, quadratic form and normaliser"}
        # algorithmic work of the particle kernel: the FP64 quadratic form c - 2 w.b + w^T A w, 2 (d^2 + d)
        # FLOP per particle (the prior draw is not counted, as for the row-by-row line)
        flop_per_launch = 2 * (d * d + d) * N
        peak, bound, unit, dtype = FP64_VALU_TFLOPS, "alu", "TFLOP/s", "f64"
    elif args.config == "mcmc-poly":
        D, C, T, burn, seed = 100, args.particles or (1 << 16), 1000, 200, 1
        x, y = synthetic.poly_data(D=D)
        dx, dy = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        data = ppl.make_data(dx, dy)
        model, kname = ppl.PPL_MODEL_POLY, "mcmc_poly_kernel"
        N = C
        workload = {"workload": "mcmc-poly", "model": "polynomial fit, lightweight Metropolis-Hastings",
                    "points": D, "chains": C, "iterations": T, "burn_in": burn, "precision": "fp64"}
        # the proposal's likelihood per iteration: 4 FMA Horner + sub + FMA square per point = 10 FLOP
        flop_per_launch = 10 * D * C * T
        peak, bound, unit, dtype = FP64_VALU_TFLOPS, "alu", "TFLOP/s", "f64"
    elif args.config == "lgssm":
        T, N, seed = 1000, args.particles or (1 << 20), 1
        y = synthetic.lgssm_data(T=T)
        dy = torch.from_numpy(y).to(dev)
        data = ppl.make_data(None, dy, dtype=ppl.PPL_F32)
        model, kname = ppl.PPL_MODEL_LGSSM, "smc_persistent_kernel"
        D = T
        workload = {"workload": "lgssm-smc", "model": "1-D linear-Gaussian state space, bootstrap SMC",
                    "steps": T, "particles": N, "ess_threshold": args.ess_frac,
                    "precision": "fp32 state, fp64 normaliser"}
        # VALU work per particle-step: 1/4 Philox block (~10 rounds of 2 mul_hi + 2 mul_lo + 4 xor/add = 20),
        # 1/2 Box-Muller pair (~12), dynamics + observation density (~6), trigger exp + sums (~4): ~42 ops
        flop_per_launch = 42 * N * T
        peak, bound, unit, dtype = FP32_VALU_UNPACKED_TFLOPS / 2, "alu", "TOP/s", "f32"
    elif args.config in ("poly", "poly-paper"):
        D = 100
        N = 10_000 if args.config == "poly" else 2_000_000
        seed = 1
        x, y = synthetic.poly_data(D=D)
        dx, dy = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
        data = ppl.make_data(dx, dy)
        model, kname = ppl.PPL_MODEL_POLY, "poly_is_kernel"
        nsum = 29
        workload = {"workload": "poly-importance-sampling", "model": "polynomial fit (degree ~ U{2..5})",
                    "points": D, "particles": N, "precision": "fp64"}
        flop_per_launch = 10 * N * D      # 4 FMA Horner + sub + FMA square, zero-padded: 10 FLOP
        peak, bound, unit, dtype = FP64_VALU_TFLOPS, "alu", "TFLOP/s", "f64"
    elif args.config == "gmm-batched":
        insts = synthetic.gmm_instances(256)
        N, seed = 1 << 16, 1
        ys = [torch.from_numpy(I["y"]).to(dev) for I in insts]
        table = ppl.InstanceTable(ys, [I["K"] for I in insts], N)
        D = sum(I["D"] for I in insts)
        kD = sum(I["D"] * I["K"] for I in insts)
        model, kname = ppl.PPL_MODEL_GMM, "smc_batched_kernel"
        workload = {"workload": "gmm-batched-smc", "model": "Gaussian mixtures, K in 3..8, batched SMC",
                    "instances": len(insts), "particles_per_instance": N, "total_data": D,
                    "max_data": max(I["D"] for I in insts), "precision": "fp32 state, fp64 normaliser"}
        # FP32 issue slots per particle-datum, transcendentals at two (their measured half rate): per
        # component 2 FMA (shifted square), max, exponent scale, v_exp (2), accumulate = 7; per datum
        # v_log (2) + scale + log-weight update = 4, and the ESS trigger: exponent, v_exp (2), 2 sums = 5
        flop_per_launch = N * (7 * kD + 9 * D)
        peak, bound, unit, dtype = FP32_VALU_UNPACKED_TFLOPS / 2, "alu", "TOP/s", "f32"

    scal = torch.empty(8, dtype=torch.float64, device=dev)
    if args.config == "gmm-batched":
        ws = ppl.workspace(ppl.ppl_smc_batched_workspace_size(model, table, None), dev)
        outb = torch.empty((table.n, 4), dtype=torch.float64, device=dev)
        tuned = ppl.ppl_smc_autotune(model, table, seed, 0.5, ws=ws, stream=stream, out=outb)
        workload["tuned"] = {"particles_per_lane": tuned[0], "wgs_per_instance": tuned[1], "spec_block": tuned[2]}

        def step():
            ppl.ppl_smc_batched(model, table, seed, 0.5, tune=tuned + (0,), ws=ws, stream=stream, out=outb)
    elif args.config == "mcmc-poly":
        ws = ppl.workspace(ppl.ppl_workspace_size(model, data, C, ppl.PPL_ALGO_MCMC), dev)
        summ = torch.empty(29, dtype=torch.float64, device=dev)

        def step():
            ppl.ppl_mcmc(model, data, C, T, seed, burn_in=burn, ws=ws, stream=stream, scalars=scal, summaries=summ)
    elif args.config == "lgssm":
        ws = ppl.workspace(ppl.ppl_workspace_size(model, data, N, ppl.PPL_ALGO_SMC), dev)

        def step():
            ppl.ppl_smc(model, data, N, seed, args.ess_frac, ws=ws, stream=stream, scalars=scal)
    else:
        ws = ppl.workspace(ppl.ppl_workspace_size(model, data, N, ppl.PPL_ALGO_IS), dev)
        summ = torch.empty(nsum, dtype=torch.float64, device=dev)

        def step():
            ppl.ppl_importance(model, data, N, seed, ws=ws, stream=stream, scalars=scal, summaries=summ)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ppl.ppl_timing_enable(True)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        step()
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    k_ms, k_n = ppl.ppl_timing_query(kname)
    ppl.ppl_timing_enable(False)
    ms_per_step = total_ms / args.steps
    evals = N * D * (T if args.config == "mcmc-poly" else 1)
    value = evals / (ms_per_step / 1e3)
    k_avg_ms = k_ms / max(k_n, 1)
    achieved = flop_per_launch / (k_avg_ms / 1e3) / (1e9 if unit == "GB/s" else 1e12)
    if args.config == "gmm-batched":
        ob = outb.cpu().numpy()
        assert (ob[:, 3] == 0).all(), "device status"
        s = [float(ob[:, 0].sum()), float(ob[:, 1].mean()), float(ob[:, 2].sum()), 0.0]
        evals = N * D
        # work counters of one more run (outside the timed steps): factors evaluated in first passes and
        # recomputed after rollbacks, against the algorithmic N D
        cnt = torch.zeros(4, dtype=torch.int64, device=dev)
        ppl.ppl_smc_batched(model, table, seed, 0.5, tune=tuned + (0,), ws=ws, stream=stream, out=outb, counters=cnt)
        c = [int(v) for v in cnt.cpu().numpy()]
        workload["work_counters"] = {"particle_factors_first_pass": c[0], "particle_factors_recomputed": c[1],
                                     "speculative_blocks": c[2], "resampling_events": c[3],
                                     "algorithmic_particle_factors": N * D,
                                     "first_pass_over_algorithmic": round(c[0] / (N * D), 4),
                                     "recomputed_over_algorithmic": round(c[1] / (N * D), 4)}
    else:
        s = scal.cpu().numpy()
        assert s[3] == 0 and math.isfinite(s[0]), f"device status {s[3]}"

    roofline = {"bound": bound, "achieved": round(achieved, 3), "peak": round(peak, 2), "unit": unit,
                "frac": round(achieved / peak, 4), "traffic": measured_traffic(args.config),
                "kernel": kname, "kernel_ms": round(k_avg_ms, 4), "kernel_launches": k_n,
                "flop_per_launch": flop_per_launch}
    if args.config == "blr":
        roofline["peak_note"] = ("peak is MI355X's published FP32 vector rate, which counts packed FP32; the "
                                 "library is compiled without packed FP32, so its attainable ceiling is the unpacked "
                                 "FMA issue rate 256 CU x 64 lanes x 2 FLOP x 2.4 GHz = 78.64 TFLOP/s")
        roofline["peak_attainable"] = round(FP32_VALU_UNPACKED_TFLOPS, 2)
        roofline["frac_attainable"] = round(achieved / FP32_VALU_UNPACKED_TFLOPS, 4)

    out = {"metric": "particle-likelihood evals/s", "value": value, "unit": "evals/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded generators, inputs resident in HBM)", "config": workload,
           "log_evidence": float(s[0]), "ess": float(s[1]), "roofline": roofline}
    if args.config == "lgssm":
        out["n_resample"] = int(s[2])
        out["metric"] = "particle-step evals/s"
    if args.config == "mcmc-poly":
        out["metric"], out["unit"], out["value"] = "MH iterations/s", "chain-iterations/s", C * T / (ms_per_step / 1e3)
        out["evals_equivalent"] = value
        out["accept_rate"] = float(s[0])
        out.pop("log_evidence"), out.pop("ess")
    if args.config == "blr-stats":
        # the statistics replace the per-row loop: the rate is in particles, not (particle, row) terms
        out["metric"], out["unit"], out["value"] = "particles/s", "particles/s", N / (ms_per_step / 1e3)
        out["evals_equivalent"] = value
    if not args.no_cpu:
        if args.config == "blr":
            out["cpu_baseline"] = cpu_baseline_blr(X, y, N, seed, target_s=args.cpu_seconds)
        elif args.config == "mcmc-poly":
            out["cpu_baseline"] = cpu_baseline_mcmc(x, y, C, T, burn, seed, target_s=args.cpu_seconds)
        elif args.config == "blr-stats":
            cb = cpu_baseline_blr(X, y, N, seed, target_s=args.cpu_seconds)
            for k in ("value", "value_1_thread"):
                cb[k] /= D                      # the oracle's row-by-row likelihood, per particle
            cb["unit"] = "particles/s"
            out["cpu_baseline"] = cb
        elif args.config == "lgssm":
            out["cpu_baseline"] = cpu_baseline_lgssm(y, seed, target_s=args.cpu_seconds)
        else:
            out["cpu_baseline"] = cpu_baseline_poly(x, y, min(N, 1 << 20), seed, target_s=args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
