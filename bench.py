"""Benchmark: k-point eigensolves/s of the per-k generalized Hermitian
eigensolve (Band_DFT_Col Parts 2-4) on one MI355X.

One step = one call of kgev_solve_k_device on a batch of nk k-points of the
magnetite-like LCAO workload (n = 2000, 16 k-points of the 4x4x4 grid,
complex128, all eigenpairs), inputs resident in HBM, kernels launched one by
one.  Prints ONE JSON line.

Extra fields:
  roofline      dominant kernel timed by HIP events carried in the dispatch
                of every --time-stride-th of its launches (the library's
                extended launch; the events are stamped when the kernel starts
                and ends, on the stream it is enqueued on), over the timed
                steps;
  roofline_gemm the complex products on FP64 MFMA timed the same way over one
                untimed step after the timed region (algorithmic flops,
                8 m n k per complex product);
  graph_replay  the same batch with the whole solve captured once as a HIP
                graph and replayed (the kernels are the same; host launch
                work disappears);
  cpu_baseline  the plain FP64 oracle on a bounded sample of the same work
                (one of the k-points), timed on the host cores, plus one
                single-threaded k-point at --cpu-single-n and the host model;
  latency_ms    p50/p99 of single-k-point calls (nk = 1, kernel by kernel);
  latency_n128_ms
                p50/p99 of single calls on the dense n = 128 pencil;
  serving       the request loop on a stream of --serve requests (n
                log-uniform in [256, --serve-nmax], 1..16 k-points) at 80% of
                its closed-loop saturation rate: p50/p99 latency, solves/s;
  fp32_refine, cholesky_s
                the mixed-precision form and the Cholesky form of Part 2 on
                the same batch (kernel by kernel), with their residuals;
  eigenvalues_only
                the same batch without eigenvectors (Band_DFT_Col's first
                pass: Part 4's tridiagonal step by bisection);
  other_workloads
                the batched-k workload (n = 1024, the 64 k-points of the 4x4x4
                grid in one call, autotuned) and the mixed-precision workload
                (n = 4096, 8 k-points, FP64 and FP32+refine), a few calls each;
  x_reuse       the batch with Part 2's X(k) exported by an earlier call and
                reused (an SCF iteration after the first: S(k) unchanged);
  host_path     the host-pointer entry point (kgev_solve_k) on the same batch
                from pageable host memory: solves/s including the PCIe
                copies, and the plain host-to-device and device-to-host copy
                times of the inputs and outputs (not the headline);
  check         residuals of one k-point and its eigenvalue error against the
                oracle's.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "k-point eigensolves/s at n=2000 (FP64 vs FP32+refine); p50/p99 latency"
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(HERE, "profiles", "hetrd_zhemv_n2000_nk16_traffic.md")
MFMA_FILE = os.path.join(HERE, "profiles", "cgemm_n2000_nk16_mfma_counters.md")
CSRC = os.path.join(HERE, "paper_1402_4247_amd", "csrc")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def zhemv_source_sha256():
    """SHA-256 of the Hermitian-product kernels' own source text (the
    hetrd_zhemv and hetrd_zhemv_tile templates in hetrd.hip, each from its
    template line to its closing brace) followed by common.hpp and lanes.hpp,
    whose helpers they use; None if a kernel is not found."""
    import hashlib
    with open(os.path.join(CSRC, "hetrd.hip")) as fh:
        text = fh.read()
    h = hashlib.sha256()
    for name in (" void hetrd_zhemv(", " void hetrd_zhemv_tile("):
        k = text.find(name)
        if k < 0:
            return None
        i0 = text.rfind("template <", 0, k)
        i1 = text.find("\n}\n", k)
        if i0 < 0 or i1 < 0:
            return None
        h.update(text[i0:i1 + 3].encode())
    for hdr in ("common.hpp", "lanes.hpp"):
        with open(os.path.join(CSRC, hdr), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def gemm_source_sha256():
    """SHA-256 of gemm.hip followed by common.hpp (the complex-product kernel
    and the helpers it uses)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("gemm.hip", "common.hpp"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def summary_fields(path):
    """The `key: value` lines of a committed counter summary."""
    fields = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    return fields


def counter_mfma(n, nk):
    """FP64 MFMA work rate of the complex products from the committed
    rocprofv3 counter summary, or None when the workload differs or the
    product kernel's source has changed since the counters were taken."""
    if (n, nk) != (2000, 16) or not os.path.exists(MFMA_FILE):
        return None
    fields = summary_fields(MFMA_FILE)
    if fields.get("source_sha256") != gemm_source_sha256():
        return None
    return {"tflops": float(fields["mfma_tflops"]), "frac": float(fields["mfma_frac"]),
            "counters": fields.get("counters"), "source": os.path.relpath(MFMA_FILE, HERE)}


def counter_traffic(n, nk):
    """HBM bytes per launch of the Hermitian-product kernel from the committed
    rocprofv3 counter summary, or None when the workload differs or the
    kernel's source has changed since the counters were taken."""
    if (n, nk) != (2000, 16) or not os.path.exists(TRAFFIC_FILE):
        return None
    fields = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if ":" in line:
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
    if fields.get("source_sha256") != zhemv_source_sha256():
        return None
    return {"bytes": float(fields["traffic_bytes_per_launch"]), "counters": fields.get("counters"),
            "ratio_to_algorithmic": float(fields["ratio_to_algorithmic"])}


def host_cpu_model():
    """The host CPU's model name and logical CPU count (from /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            names = [l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")]
        return {"model": names[0] if names else None, "logical_cpus": len(names), "affinity": len(os.sched_getaffinity(0))}
    except OSError:
        return None


def roofline_object(prof, phase, elapsed, note, traffic, K):
    """Roofline object of one phase from the library's sampled launch timing:
    achieved = algorithmic work per timed launch / mean timed duration."""
    hemv = phase == K.PHASE_HEMV
    # the Hermitian product of a blocked column runs in one of two forms,
    # four 64 x 64 tiles per workgroup (hetrd_zhemv) or one (hetrd_zhemv_tile),
    # chosen per column by the workgroup count: the phase covers both
    base = {"bound": "hbm" if hemv else "mfma",
            "kernel": "hetrd_zhemv + hetrd_zhemv_tile" if hemv else "cgemm_kernel",
            "peak": PEAK_HBM_GBS if hemv else PEAK_FP64_TFLOPS, "unit": "GB/s" if hemv else "TFLOP/s"}
    if prof is None:
        return {**base, "achieved": None, "frac": None, "traffic": None,
                "measured_on": "not measured (kernel timing off)"}
    if prof["launches"] == 0:
        # at orders up to 128 the LDS-resident tail kernel reduces the whole
        # matrix, so there is no Hermitian-product launch
        return {**base, "achieved": None, "frac": None, "traffic": None, "launches": 0, "timed_launches": 0,
                "measured_on": "no launch of the kernel at this order", "share_of_step": 0.0}
    avg_ms = prof["ms"] / prof["launches"]
    share = avg_ms * prof["phase_launches"] / (1e3 * elapsed)
    if hemv:
        per_launch = prof["bytes"] / prof["launches"]
        achieved = per_launch / (avg_ms * 1e-3) / 1e9
        extra = {"alg_bytes_per_launch": per_launch}
    else:
        per_launch = prof["flops"] / prof["launches"]
        achieved = per_launch / (avg_ms * 1e-3) / 1e12
        extra = {"alg_flops_per_launch": per_launch,
                 "flop_count": "8 m n k per complex product (half for lower-only outputs, 4 m n k for a real "
                               "right operand), whatever the kernel's own form"}
    if traffic is not None:
        extra["traffic_counters"] = traffic["counters"]
        extra["traffic_ratio_to_algorithmic"] = traffic["ratio_to_algorithmic"]
    return {**base, "achieved": achieved, "frac": achieved / base["peak"],
            "traffic": None if traffic is None else traffic["bytes"],
            "launches": prof["phase_launches"], "timed_launches": prof["launches"], "avg_launch_us": 1e3 * avg_ms,
            **extra, "measured_on": note, "share_of_step": share}


def serve_stream(args, K, G, torch, dev):
    """Serving workload: requests with n log-uniform in [256, nmax] (the order
    taken at the centre of one of --serve-bins equal bins of log n, so the
    pool's mean cost matches the continuous distribution's) and 1..16
    k-points, arriving as a Poisson process at 80% of the closed-loop
    saturation rate of the same mix.  Each pool order has one seeded LCAO
    pencil, replicated over the request's k-points (the cost of a k-point
    does not depend on which k it is)."""
    import math
    rng = np.random.default_rng(5005)
    lo, hi, nb = math.log(256), math.log(args.serve_nmax), args.serve_bins
    sizes = sorted({int(round(math.exp(lo + (i + 0.5) * (hi - lo) / nb))) for i in range(nb)})
    log(f"[serve] pool orders {sizes}")
    pool = {}
    for n in sizes:
        Hs, Ss = G.lcao_batch(n, G.mp_grid(4)[:1], 5005 + n)
        dH = torch.from_numpy(G.colmajor(Hs)).to(dev).expand(16, n, n).contiguous()
        dS = torch.from_numpy(G.colmajor(Ss)).to(dev).expand(16, n, n).contiguous()
        pool[n] = (dH, dS)
    reqs = [(sizes[int(rng.integers(0, len(sizes)))], int(rng.integers(1, 17))) for _ in range(args.serve)]

    # results are collected oldest first once more than this many requests
    # (or this many output bytes) are outstanding, so long streams fit in HBM;
    # the server stamps completion itself, so late collection does not
    # change the measured latency
    max_inflight, max_bytes = 48, 64 << 30
    budget = 140 << 30          # the server's workspace budget; inputs and outputs live beside it

    def run(arrivals, what, reqs=reqs):
        from collections import deque
        res = [None] * len(reqs)
        with K.Server(0, budget, args.serve_slots) as srv:
            t0 = time.perf_counter()
            inflight = deque()
            held = 0
            collected = 0

            def collect():
                nonlocal held, collected
                idx, t, nbytes, _outs = inflight.popleft()
                res[idx] = srv.wait(t)
                held -= nbytes
                collected += 1
                if collected % 25 == 0:
                    log(f"[serve] {what}: {collected}/{len(reqs)} requests done")

            for idx, ((n, nk), ta) in enumerate(zip(reqs, arrivals)):
                delay = t0 + ta - time.perf_counter()
                if delay > 0:
                    time.sleep(delay)
                nbytes = nk * n * n * 16 + nk * n * 8
                while inflight and (len(inflight) >= max_inflight or held + nbytes > max_bytes):
                    collect()
                w = torch.empty((nk, n), dtype=torch.float64, device=dev)
                C = torch.empty((nk, n, n), dtype=torch.complex128, device=dev)
                dH, dS = pool[n]
                # the output tensors stay referenced until the request is collected
                inflight.append((idx, srv.submit(dH, dS, n, nk, w, C), nbytes, (w, C)))
                held += nbytes
            while inflight:
                collect()
            t1 = time.perf_counter()
        return res, t1 - t0

    # closed loop (everything queued at t = 0) gives the saturation rate, on
    # the first --serve-sat requests of the stream (all of them by default)
    nsat = min(len(reqs), args.serve_sat) if args.serve_sat > 0 else len(reqs)
    log(f"[serve] closed loop, {nsat} requests")
    res, span = run([0.0] * nsat, "closed loop", reqs[:nsat])
    sat = nsat / span
    lam = 0.8 * sat
    gaps = rng.exponential(1.0 / lam, len(reqs))
    arrivals = np.cumsum(gaps) - gaps[0]
    log(f"[serve] open loop at {lam:.2f} requests/s")
    res, span = run(list(arrivals), "open loop")
    lat = np.array([1e3 * (r.t_done - r.t_submit) for r in res])
    solves = sum(nk for _, nk in reqs)
    return {"requests": len(reqs), "slots": args.serve_slots, "orders": sizes,
            "saturation_requests": nsat, "saturation_requests_per_s": sat, "arrival_rate_requests_per_s": lam,
            "solves_per_s": solves / span, "latency_ms_p50": float(np.percentile(lat, 50)),
            "latency_ms_p99": float(np.percentile(lat, 99)),
            "status_all_ok": all(r.status == 0 for r in res)}


def device_residuals(torch, dH, dS, dw, dC, k):
    """r_res and max |C^H S C - I| of k-point k with torch products on the
    device (column-major buffers)."""
    H = dH[k].transpose(0, 1).contiguous()
    S = dS[k].transpose(0, 1).contiguous()
    C = dC[k].transpose(0, 1).contiguous()
    SC = S @ C
    R = H @ C - SC * dw[k].to(torch.complex128)[None, :]
    r_res = float(torch.linalg.matrix_norm(R) / torch.linalg.matrix_norm(H))
    CSC = C.conj().transpose(0, 1).contiguous() @ SC
    r_orth = float((CSC - torch.eye(C.shape[0], dtype=torch.complex128, device=C.device)).abs().max())
    return r_res, r_orth


def other_configs(args, K, G, torch, dev, ctx):
    """The batched-k workload (n = 1024, the 64 k-points of the 4x4x4 grid,
    autotuned) and the mixed-precision workload (n = 4096, the 8 k-points of
    the 2x2x2 grid, FP64 and complex64 reduction + FP64 refinement), a few
    timed calls each after one untimed call."""
    out = {}

    def timed(n, nk, dH, dS, opts, steps):
        dw = torch.zeros((nk, n), dtype=torch.float64, device=dev)
        dC = torch.zeros((nk, n, n), dtype=torch.complex128, device=dev)
        st = torch.zeros(nk, dtype=torch.int32, device=dev)
        ms = []
        for r in range(steps + 1):
            torch.cuda.synchronize()
            a = time.perf_counter()
            rc = K.solve_k_device(ctx, dH, dS, n, n, nk, dw, dC, n, d_status=st, opts=opts)
            torch.cuda.synchronize()
            if rc != 0:
                raise RuntimeError(f"solve n={n} nk={nk} returned {rc}")
            if r >= 1:
                ms.append(1e3 * (time.perf_counter() - a))
        return dw, dC, st, float(np.mean(ms))

    if args.config3_steps > 0:
        n, nk = 1024, 64
        log(f"[bench] batched-k workload n={n} nk={nk}: generating, autotuning")
        Hs, Ss = G.config3(n, nk, 3003)
        dH = torch.from_numpy(G.colmajor(Hs)).to(dev)
        dS = torch.from_numpy(G.colmajor(Ss)).to(dev)
        del Hs, Ss
        nb = K.autotune(ctx, n)
        _, hs, gs, _ = K.tuned_params(ctx, n)
        dw, dC, st, ms = timed(n, nk, dH, dS, K.make_opts(), args.config3_steps)
        r_res, r_orth = device_residuals(torch, dH, dS, dw, dC, 0)
        out["batched_n1024_nk64"] = {
            "value": nk * 1e3 / ms, "unit": "solves/s", "ms_per_call": ms, "calls": args.config3_steps,
            "workload": "LCAO pencil n=1024, the 64 k-points of the 4x4x4 grid in one call, seed 3003",
            "tuned": {"panel_nb": nb, "hemv_slots": hs, "gemm_slots": gs},
            "status_all_ok": bool(np.all(st.cpu().numpy() == 0)), "r_res_k0": r_res, "r_orth_k0": r_orth}
        log(f"[bench] batched-k workload {out['batched_n1024_nk64']['value']:.1f} solves/s")
        del dH, dS, dw, dC
    if args.config4_steps > 0:
        n, nk = 4096, 8
        log(f"[bench] mixed-precision workload n={n} nk={nk}: generating")
        Hs, Ss = G.config4(n, nk, 4004)
        dH = torch.from_numpy(G.colmajor(Hs)).to(dev)
        dS = torch.from_numpy(G.colmajor(Ss)).to(dev)
        del Hs, Ss
        dw, dC, st, ms = timed(n, nk, dH, dS, K.make_opts(), args.config4_steps)
        r_res, r_orth = device_residuals(torch, dH, dS, dw, dC, 0)
        w64 = dw.cpu().numpy()
        ok64 = bool(np.all(st.cpu().numpy() == 0))
        del dC
        dwm, dCm, stm, msm = timed(n, nk, dH, dS, K.make_opts(precision=K.PREC_FP32_REFINE), args.config4_steps)
        rm_res, rm_orth = device_residuals(torch, dH, dS, dwm, dCm, 0)
        wm = dwm.cpu().numpy()
        out["mixed_n4096_nk8"] = {
            "workload": "LCAO pencil n=4096, the 8 k-points of the 2x2x2 grid in one call, seed 4004",
            "fp64": {"value": nk * 1e3 / ms, "unit": "solves/s", "ms_per_call": ms, "calls": args.config4_steps,
                     "status_all_ok": ok64, "r_res_k0": r_res, "r_orth_k0": r_orth},
            "fp32_refine": {"value": nk * 1e3 / msm, "unit": "solves/s", "ms_per_call": msm,
                            "calls": args.config4_steps, "status_all_ok": bool(np.all(stm.cpu().numpy() == 0)),
                            "r_res_k0": rm_res, "r_orth_k0": rm_orth,
                            "eig_diff_vs_fp64_rel": float(np.abs(wm - w64).max() / np.abs(w64).max())}}
        log(f"[bench] mixed-precision workload: fp64 {nk * 1e3 / ms:.2f}, fp32+refine {nk * 1e3 / msm:.2f} solves/s")
        del dH, dS, dwm, dCm
    torch.cuda.empty_cache()
    return out or None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=2000)
    ap.add_argument("--nk", type=int, default=16)
    ap.add_argument("--seed", type=int, default=2002)
    ap.add_argument("--generator", choices=["lcao", "dense"], default="lcao",
                    help="lcao: the magnetite-like LCAO pencils (k-point batch); dense: independent dense "
                         "well-conditioned pencils, S = I + 0.05 (A + A^H)/2 and H = Q diag(l) Q^H")
    ap.add_argument("--roofline-phase", choices=["hemv", "gemm"], default="hemv")
    ap.add_argument("--time-stride", type=int, default=17,
                    help="time every N-th launch of the roofline kernel with HIP events")
    ap.add_argument("--kernel-timing", choices=["on", "off"], default="on",
                    help="off: no launch carries timing events (for runs under a counter-collecting "
                         "profiler); the roofline objects are then null")
    ap.add_argument("--gemm-steps", type=int, default=1,
                    help="untimed steps after the timed region whose complex products are timed for the "
                         "second roofline object (0 skips it)")
    ap.add_argument("--latency128-reps", type=int, default=200,
                    help="single-pencil latency of the dense n = 128 pencil (seed 1001), repetitions (0 skips)")
    ap.add_argument("--cpu-single-n", type=int, default=1024,
                    help="order of the single-threaded oracle sample (0 skips it)")
    ap.add_argument("--latency-reps", type=int, default=50, help="0 skips the latency measurement")
    ap.add_argument("--reuse-steps", type=int, default=2,
                    help="timed calls reusing Part 2's X from an earlier call (0 skips them)")
    ap.add_argument("--host-steps", type=int, default=1,
                    help="timed calls of the host-pointer entry point (0 skips it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-steps", type=int, default=2,
                    help="timed steps of the FP32+refine form (0 skips it)")
    ap.add_argument("--values-steps", type=int, default=2,
                    help="timed steps of the eigenvalues-only solve (Band_DFT_Col's first pass; 0 skips it)")
    ap.add_argument("--cholesky-steps", type=int, default=2,
                    help="steps of the Cholesky form of Part 2 on the same batch (0 skips it)")
    ap.add_argument("--serve", type=int, default=64,
                    help="also run the serving stream with this many requests (0 skips it)")
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--config3-steps", type=int, default=3,
                    help="timed calls of the batched-k workload (n=1024, 64 k-points, autotuned; 0 skips it)")
    ap.add_argument("--config4-steps", type=int, default=2,
                    help="timed calls of the mixed-precision workload (n=4096, 8 k-points, FP64 and "
                         "FP32+refine; 0 skips it)")
    ap.add_argument("--serve-bins", type=int, default=6,
                    help="pool orders: the centres of this many equal bins of log n in [256, --serve-nmax]")
    ap.add_argument("--serve-sat", type=int, default=0,
                    help="requests of the closed-loop run that measures the saturation rate (0: all)")
    ap.add_argument("--serve-nmax", type=int, default=2000)
    ap.add_argument("--panel-nb", type=int, default=0,
                    help="Householder panel width (0: the library default, or the tuned width with --autotune)")
    ap.add_argument("--hemv-slots", type=int, default=0,
                    help="Hermitian-product tile grouping threshold (opts.hemv_slots; 0: tuned or default)")
    ap.add_argument("--gemm-slots", type=int, default=0,
                    help="product tile threshold (opts.gemm_slots; 0: tuned or default)")
    ap.add_argument("--graph-steps", type=int, default=3,
                    help="steps of graph replay (the solve captured once as a HIP graph) reported beside the "
                         "kernel-by-kernel headline; 0 skips it")
    ap.add_argument("--autotune", action="store_true",
                    help="run kgev_autotune for this n before timing (the tuned panel width and "
                         "Hermitian-product threshold are then used)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="run only a plain device-to-device copy of MIB MiB (3 launches) and exit: the "
                         "reference of known size for scaling the HBM byte counters")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the per-k solve needs no "
                                   "communication, and a multi-GPU run would give each GPU its own "
                                   "share of the k-points",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    if args.copy_calib > 0:
        nbytes = args.copy_calib << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calib_bytes_read": nbytes, "copy_calib_bytes_written": nbytes, "launches": 3}))
        return
    from paper_1402_4247_amd import inputs as G
    from paper_1402_4247_amd import kgev as K

    n, nk = args.n, args.nk
    log(f"[bench] generating workload n={n} nk={nk}")
    Hs, Ss = G.config2(n, nk, args.seed) if args.generator == "lcao" else G.config1_batch(n, nk, args.seed)
    dev = torch.device("cuda:0")
    dH = torch.from_numpy(G.colmajor(Hs)).to(dev)
    dS = torch.from_numpy(G.colmajor(Ss)).to(dev)
    dw = torch.zeros((nk, n), dtype=torch.float64, device=dev)
    dC = torch.zeros((nk, n, n), dtype=torch.complex128, device=dev)
    dst = torch.zeros(nk, dtype=torch.int32, device=dev)
    opts = K.make_opts(panel_nb=args.panel_nb, hemv_slots=args.hemv_slots, gemm_slots=args.gemm_slots)
    ctx = K.Context(0)
    tuned_nb = None
    if args.autotune:
        tuned_nb = K.autotune(ctx, n)
        log(f"[bench] autotuned panel width {tuned_nb}")
    _, hemv_slots, gemm_slots, _ = K.tuned_params(ctx, n)
    if args.autotune:
        log(f"[bench] autotuned thresholds: Hermitian product {hemv_slots}, products {gemm_slots} workgroups")

    def step():
        st = K.solve_k_device(ctx, dH, dS, n, n, nk, dw, dC, n, d_status=dst, opts=opts)
        if st != 0:
            raise RuntimeError(f"kgev_solve_k_device returned {st}")

    log(f"[bench] warmup {args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    phase = K.PHASE_HEMV if args.roofline_phase == "hemv" else K.PHASE_GEMM
    timing = args.kernel_timing == "on"
    if timing:
        K.profile_begin(ctx, phase, args.time_stride)
    log(f"[bench] timing {args.steps} steps")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    marks = []
    for _ in range(args.steps):
        step()
        torch.cuda.synchronize()      # per-step times for the median; the GPU idles only between calls
        marks.append(time.perf_counter())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms = np.diff(np.array([t0] + marks)) * 1e3
    prof = K.profile_end(ctx) if timing else None
    elapsed = t1 - t0
    ms_per_step = 1e3 * elapsed / args.steps
    value = nk * args.steps / elapsed
    status = dst.cpu().numpy()
    log(f"[bench] {ms_per_step:.1f} ms/step, {value:.2f} solves/s, status {set(status.tolist())}")
    note = (f"every {args.time_stride}-th launch of the timed steps" if args.time_stride > 1
            else "every launch of the timed steps")
    roof = roofline_object(prof, phase, elapsed, note, counter_traffic(n, nk) if phase == K.PHASE_HEMV else None, K)

    # the other phase (the complex products on MFMA, or the Hermitian
    # product), timed the same way over untimed steps after the timed region
    roof2 = None
    if timing and args.gemm_steps > 0:
        ph2 = K.PHASE_GEMM if phase == K.PHASE_HEMV else K.PHASE_HEMV
        K.profile_begin(ctx, ph2, args.time_stride)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.gemm_steps):
            step()
        torch.cuda.synchronize()
        el2 = time.perf_counter() - a
        prof2 = K.profile_end(ctx)
        roof2 = roofline_object(prof2, ph2, el2, f"every {args.time_stride}-th launch of {args.gemm_steps} "
                                "untimed step(s) after the timed region", None, K)
        mc = counter_mfma(n, nk)
        if mc is not None:
            roof2["mfma_counters"] = mc
        log(f"[bench] second roofline: {roof2['kernel']} {roof2['achieved']} {roof2['unit']}")

    # latency of single-k-point calls
    lat = []
    reps_total = args.latency_reps + 2 if args.latency_reps > 0 else 0
    w1 = torch.zeros((1, n), dtype=torch.float64, device=dev)
    C1 = torch.zeros((1, n, n), dtype=torch.complex128, device=dev)
    for r in range(reps_total):
        torch.cuda.synchronize()
        a = time.perf_counter()
        st = K.solve_k_device(ctx, dH[:1], dS[:1], n, n, 1, w1, C1, n, opts=opts)
        torch.cuda.synchronize()
        if st != 0:
            raise RuntimeError(f"latency call returned {st}")
        if r >= 2:
            lat.append(1e3 * (time.perf_counter() - a))
    lat = np.array(lat) if lat else np.array([float("nan")])
    log(f"[bench] latency p50 {np.percentile(lat, 50):.1f} ms p99 {np.percentile(lat, 99):.1f} ms")

    # single-pencil latency of the dense n = 128 pencil: the whole solve of
    # one small system, back-to-back calls with inputs in HBM
    lat128 = None
    if args.latency128_reps > 0:
        H1, S1 = G.config1(128, 1001)
        dH1 = torch.from_numpy(G.colmajor(H1[None])).to(dev)
        dS1 = torch.from_numpy(G.colmajor(S1[None])).to(dev)
        w128 = torch.zeros((1, 128), dtype=torch.float64, device=dev)
        C128 = torch.zeros((1, 128, 128), dtype=torch.complex128, device=dev)
        t128 = []
        for r in range(args.latency128_reps + 5):
            torch.cuda.synchronize()
            a = time.perf_counter()
            st = K.solve_k_device(ctx, dH1, dS1, 128, 128, 1, w128, C128, 128, opts=K.make_opts())
            torch.cuda.synchronize()
            if st != 0:
                raise RuntimeError(f"n = 128 latency call returned {st}")
            if r >= 5:
                t128.append(1e3 * (time.perf_counter() - a))
        t128 = np.array(t128)
        C1h = C128[0].cpu().numpy().T
        w1h = w128[0].cpu().numpy()
        lat128 = {"p50": float(np.percentile(t128, 50)), "p99": float(np.percentile(t128, 99)), "reps": int(t128.size),
                  "workload": "dense pencil n = 128 (S = I + 0.05 (A + A^H)/2, H = Q diag(l) Q^H, seed 1001), nk = 1",
                  "r_res": float(np.linalg.norm(H1 @ C1h - S1 @ C1h * w1h) / np.linalg.norm(H1)),
                  "r_orth": float(np.abs(C1h.conj().T @ S1 @ C1h - np.eye(128)).max())}
        log(f"[bench] n = 128 latency p50 {lat128['p50']:.3f} ms p99 {lat128['p99']:.3f} ms")

    # accuracy of k-point 0 of the timed batch
    w0 = dw[0].cpu().numpy()
    C0 = dC[0].cpu().numpy().T
    H0, S0 = Hs[0], Ss[0]
    r_res = float(np.linalg.norm(H0 @ C0 - S0 @ C0 * w0) / np.linalg.norm(H0))
    r_orth = float(np.abs(C0.conj().T @ S0 @ C0 - np.eye(n)).max())
    check = {"k": 0, "r_res": r_res, "r_orth": r_orth, "status_all_ok": bool(np.all(status == 0))}

    # the mixed-precision form on the same batch, same accuracy gate
    mixed = None
    if args.mixed_steps > 0:
        om = K.make_opts(precision=K.PREC_FP32_REFINE)
        wm = torch.zeros_like(dw)
        Cm = torch.zeros_like(dC)
        stm = torch.zeros_like(dst)

        def mstep():
            st = K.solve_k_device(ctx, dH, dS, n, n, nk, wm, Cm, n, d_status=stm, opts=om)
            if st != 0:
                raise RuntimeError(f"mixed solve returned {st}")

        log(f"[bench] FP32+refine: warmup 1, timing {args.mixed_steps} steps")
        mstep()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.mixed_steps):
            mstep()
        torch.cuda.synchronize()
        tm = time.perf_counter() - a
        wmk = wm[0].cpu().numpy()
        Cmk = Cm[0].cpu().numpy().T
        mixed = {"value": nk * args.mixed_steps / tm, "unit": "solves/s",
                 "ms_per_step": 1e3 * tm / args.mixed_steps, "steps": args.mixed_steps,
                 "refine_sweeps": 3, "status_all_ok": bool(np.all(stm.cpu().numpy() == 0)),
                 "r_res": float(np.linalg.norm(H0 @ Cmk - S0 @ Cmk * wmk) / np.linalg.norm(H0)),
                 "r_orth": float(np.abs(Cmk.conj().T @ S0 @ Cmk - np.eye(n)).max()),
                 "eig_diff_vs_fp64_rel": float(np.abs(wmk - w0).max() / np.abs(w0).max())}
        log(f"[bench] FP32+refine {mixed['value']:.2f} solves/s")

    # Band_DFT_Col's eigenvalue pass: the same batch without eigenvectors
    # (Part 4's tridiagonal step by bisection)
    values = None
    if args.values_steps > 0:
        ov = K.make_opts(want_vectors=False)
        wv = torch.zeros_like(dw)
        stv = torch.zeros_like(dst)

        def vstep():
            st = K.solve_k_device(ctx, dH, dS, n, n, nk, wv, None, n, d_status=stv, opts=ov)
            if st != 0:
                raise RuntimeError(f"eigenvalues-only solve returned {st}")

        log(f"[bench] eigenvalues only: warmup 1, timing {args.values_steps} steps")
        vstep()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.values_steps):
            vstep()
        torch.cuda.synchronize()
        tv = time.perf_counter() - a
        values = {"value": nk * args.values_steps / tv, "unit": "solves/s", "ms_per_step": 1e3 * tv / args.values_steps,
                  "steps": args.values_steps, "status_all_ok": bool(np.all(stv.cpu().numpy() == 0)),
                  "eig_diff_vs_vectors_solve_rel": float((wv - dw).abs().max().item() / dw.abs().max().item())}
        log(f"[bench] eigenvalues only {values['value']:.2f} solves/s")

    # Part 2 in Cholesky form (X = L^-H) on the same batch, same accuracy gate
    chol = None
    if args.cholesky_steps > 0:
        oc = K.make_opts(s_method=K.S_CHOLESKY)
        wc = torch.zeros_like(dw)
        Cc = torch.zeros_like(dC)
        stc = torch.zeros_like(dst)

        def cstep():
            st = K.solve_k_device(ctx, dH, dS, n, n, nk, wc, Cc, n, d_status=stc, opts=oc)
            if st != 0:
                raise RuntimeError(f"Cholesky-form solve returned {st}")

        log(f"[bench] Cholesky form: warmup 1, timing {args.cholesky_steps} steps")
        cstep()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.cholesky_steps):
            cstep()
        torch.cuda.synchronize()
        tc = time.perf_counter() - a
        wck = wc[0].cpu().numpy()
        Cck = Cc[0].cpu().numpy().T
        chol = {"value": nk * args.cholesky_steps / tc, "unit": "solves/s",
                "ms_per_step": 1e3 * tc / args.cholesky_steps, "steps": args.cholesky_steps,
                "status_all_ok": bool(np.all(stc.cpu().numpy() == 0)),
                "r_res": float(np.linalg.norm(H0 @ Cck - S0 @ Cck * wck) / np.linalg.norm(H0)),
                "r_orth": float(np.abs(Cck.conj().T @ S0 @ Cck - np.eye(n)).max()),
                "eig_diff_vs_fp64_rel": float(np.abs(wck - w0).max() / np.abs(w0).max())}
        log(f"[bench] Cholesky form {chol['value']:.2f} solves/s")

    # the same batch in graph mode: captured once (untimed), then replayed
    graph = None
    if args.graph_steps > 0:
        og = K.make_opts(panel_nb=args.panel_nb, hemv_slots=args.hemv_slots, gemm_slots=args.gemm_slots,
                         use_graph=True)
        gs = torch.cuda.Stream()
        wg = torch.zeros_like(dw)
        Cg = torch.zeros_like(dC)
        stg = torch.zeros_like(dst)

        def gstep():
            with torch.cuda.stream(gs):
                st = K.solve_k_device(ctx, dH, dS, n, n, nk, wg, Cg, n, d_status=stg, opts=og,
                                      stream=gs.cuda_stream)
            if st != 0:
                raise RuntimeError(f"graph-mode solve returned {st}")

        log(f"[bench] graph replay: capture, timing {args.graph_steps} replays")
        gstep()
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.graph_steps):
            gstep()
        torch.cuda.synchronize()
        tg = time.perf_counter() - a
        graph = {"value": nk * args.graph_steps / tg, "unit": "solves/s",
                 "ms_per_step": 1e3 * tg / args.graph_steps, "steps": args.graph_steps,
                 "bitwise_equal_to_headline": bool(torch.equal(wg, dw) and torch.equal(Cg, dC)),
                 "status_all_ok": bool(np.all(stg.cpu().numpy() == 0))}
        log(f"[bench] graph replay {graph['value']:.2f} solves/s")

    # an SCF iteration after the first: S(k) unchanged, so Part 2's X(k) from
    # an earlier call is reused and only Parts 3-4 run (same H here)
    xreuse = None
    if args.reuse_steps > 0:
        dX = torch.empty((nk, n, n), dtype=torch.complex128, device=dev)
        wx = torch.zeros_like(dw)
        Cx = torch.zeros_like(dC)
        stx = torch.zeros_like(dst)
        st = K.solve_k_x_device(ctx, dH, dS, n, n, nk, wx, Cx, n, dX, K.X_EXPORT, d_status=stx, opts=opts)
        if st != 0:
            raise RuntimeError(f"X export returned {st}")
        log(f"[bench] X reuse: timing {args.reuse_steps} calls")
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.reuse_steps):
            st = K.solve_k_x_device(ctx, dH, dS, n, n, nk, wx, Cx, n, dX, K.X_REUSE, d_status=stx, opts=opts)
            if st != 0:
                raise RuntimeError(f"X reuse returned {st}")
        torch.cuda.synchronize()
        tx = time.perf_counter() - a
        xreuse = {"value": nk * args.reuse_steps / tx, "unit": "solves/s", "ms_per_step": 1e3 * tx / args.reuse_steps,
                  "steps": args.reuse_steps, "status_all_ok": bool(np.all(stx.cpu().numpy() == 0)),
                  "bitwise_equal_to_headline": bool(torch.equal(wx, dw) and torch.equal(Cx, dC))}
        del dX, Cx
        log(f"[bench] X reuse {xreuse['value']:.2f} solves/s")

    # the host-pointer entry point: PCIe copies included
    host = None
    if args.host_steps > 0:
        Hc = np.ascontiguousarray(G.colmajor(Hs))
        Sc = np.ascontiguousarray(G.colmajor(Ss))
        wh = np.zeros((nk, n))
        Ch = np.zeros((nk, n, n), dtype=np.complex128)
        log(f"[bench] host-pointer path: warmup 1, timing {args.host_steps} calls")
        K.solve_k(ctx, Hc, Sc, n, nk, wh, Ch)
        a = time.perf_counter()
        for _ in range(args.host_steps):
            sth, _bad = K.solve_k(ctx, Hc, Sc, n, nk, wh, Ch)
            if sth != 0:
                raise RuntimeError(f"kgev_solve_k returned {sth}")
        th = (time.perf_counter() - a) / args.host_steps
        torch.cuda.synchronize()
        a = time.perf_counter()
        tH = torch.from_numpy(Hc).to(dev)
        tS = torch.from_numpy(Sc).to(dev)
        torch.cuda.synchronize()
        h2d = time.perf_counter() - a
        a = time.perf_counter()
        _ = dC.cpu()
        d2h = time.perf_counter() - a
        del tH, tS, _
        host = {"value": nk / th, "unit": "solves/s", "ms_per_call": 1e3 * th, "calls": args.host_steps,
                "h2d_ms_H_S": 1e3 * h2d, "d2h_ms_C": 1e3 * d2h,
                "bitwise_equal_to_headline": bool(np.array_equal(wh, dw.cpu().numpy()))}
        log(f"[bench] host-pointer path {host['value']:.2f} solves/s")

    serving = serve_stream(args, K, G, torch, dev) if args.serve > 0 else None
    others = other_configs(args, K, G, torch, dev, ctx)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle as O
        threads = O.max_threads()
        log(f"[bench] cpu baseline: oracle on k-point 0 with {threads} threads")
        a = time.perf_counter()
        st0, wor, _ = O.solve_k(H0, S0)
        t_or = time.perf_counter() - a
        cpu = {"value": 1.0 / t_or, "unit": "solves/s", "cores": threads, "kind": "oracle",
               "sample": f"1 of the {nk} k-points (k index 0) at n={n}, all eigenpairs; {t_or:.1f} s",
               "host_cpu": host_cpu_model()}
        check["eig_err_vs_oracle_rel"] = float(np.abs(w0 - wor).max() / np.abs(wor).max())
        if mixed is not None:
            mixed["eig_err_vs_oracle_rel"] = float(np.abs(wmk - wor).max() / np.abs(wor).max())
        check["oracle_status"] = int(st0)
        if args.cpu_single_n > 0:
            ns = args.cpu_single_n
            Hq, Sq = G.lcao_batch(ns, G.mp_grid(4)[:1], args.seed)
            log(f"[bench] cpu baseline: oracle on one k-point at n={ns} with 1 thread")
            O.set_threads(1)
            a = time.perf_counter()
            O.solve_k(Hq[0], Sq[0])
            t1t = time.perf_counter() - a
            O.set_threads(threads)
            cpu["single_thread"] = {"value": 1.0 / t1t, "unit": "solves/s", "cores": 1,
                                    "sample": f"1 k-point of the LCAO pencil at n={ns}, all eigenpairs; {t1t:.1f} s"}

    out = {
        "metric": METRIC, "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "ms_per_step_median": float(np.median(step_ms)),
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": (f"magnetite-like LCAO pencil H(k)C = S(k)C Lambda, n={n}, {nk} k-points of the "
                                "4x4x4 Monkhorst-Pack grid, complex128, all eigenpairs" if args.generator == "lcao" else
                                f"dense well-conditioned pencil H C = S C Lambda (S = I + 0.05 (A + A^H)/2, H with "
                                f"eigenvalues uniform in [-1, 1]), n={n}, {nk} independent pencils, complex128, all "
                                "eigenpairs"),
                   "n": n, "nk": nk, "precision": "fp64", "seed": args.seed,
                   "panel_nb": args.panel_nb or tuned_nb or 32, "hemv_slots": args.hemv_slots or hemv_slots,
                   "gemm_slots": args.gemm_slots or gemm_slots,
                   "autotuned": bool(args.autotune)},
        "roofline": roof, "roofline_gemm": roof2, "cpu_baseline": cpu, "graph_replay": graph, "fp32_refine": mixed, "eigenvalues_only": values, "cholesky_s": chol,
        "host_path": host, "x_reuse": xreuse, "serving": serving,
        "latency_ms": ({"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                        "reps": int(lat.size), "nk": 1} if args.latency_reps > 0 else None),
        "latency_n128_ms": lat128,
        "other_workloads": others,
        "check": check,
    }
    ctx.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
