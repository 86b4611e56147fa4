#!/usr/bin/env python3
"""Decoded Mbit/s of the Log-Fourier SP decoder on one MI355X.

Workload (default): GF(64) (2,6) code, N=1000 symbols (M=333 checks, E=2000
edges), 4096 frames of random codewords over BPSK/AWGN at Eb/N0 = 2.5 dB,
max 100 rounds, stop at zero syndrome.  One step = one complete decode of the
4096-frame batch (every round until every frame has stopped), with the LLRs
already resident in HBM.

Prints one JSON line.  `value` comes from the timed decodes as the library
runs them (graph replay of chunks of rounds).  `roofline` is measured live for
the fused pass kernel over as many further decodes of the same batch with HIP
events around each launch on the decode stream (eager launches, since kernels
inside a replayed graph cannot be timed): algorithmic bytes per frame-round
B = (2E+N)*q*s + 4*N*m (s = bytes per stored message entry), plus
E*q*s + 4*N*m for the first pass of each frame.  `cpu_baseline` times the FP64
oracle on a bounded sample of the same frames on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "decoded Mbit/s at GF(64)(2,6) N=1000, 2.5 dB; p50/p99 frame latency"
HBM_PEAK_GBS = 8000.0


def _oracle_worker(args):
    idx, llr, code_arrays, max_iter = args
    from oracle.sp import TannerCode, decode
    M, N, m, rp, col, val, poly = code_arrays
    tc = TannerCode(M, N, m, rp, col, val, poly)
    t0 = time.perf_counter()
    r = decode(tc, llr, max_iter)
    return idx, time.perf_counter() - t0, r.hard, r.iters


def host_cores():
    """Host cores this process may use: the affinity mask, capped at 16 (the
    host CPU share that goes with one GPU on the measurement machines, whatever
    the machine's total core count)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(batch, max_iter, frames_per_worker=2, workers=None):
    """Time the FP64 oracle (never tuned) on a sample of the batch's frames."""
    import multiprocessing as mp
    workers = workers or host_cores()
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ[k] = "1"
    c = batch.code
    arrays = (c.M, c.N, c.m, c.row_ptr, c.col, c.val, c.poly)
    n = workers * frames_per_worker
    sample = np.linspace(0, batch.llr.shape[0] - 1, n).astype(int)
    tasks = [(sample[i::workers], batch.llr[sample[i::workers]], arrays, max_iter) for i in range(workers)]
    ctx = mp.get_context("spawn")
    with ctx.Pool(workers) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_worker, tasks)
        wall = time.perf_counter() - t0
    frames = sum(len(r[0]) for r in res)
    mbps = frames * batch.info_bits_per_frame / wall / 1e6
    return dict(value=mbps, unit="Mbit/s", cores=workers, kind="oracle",
                sample=f"{frames} frames (evenly spaced over the batch), full decode to the same stop rule, "
                       f"{workers} processes x 1 thread (all of the host share), {wall:.1f} s wall"), res


def oracle_agreement(res, hard, iters):
    """Per-frame agreement of a GPU decode with the oracle sample: frames whose
    hard decisions and stopping round are both identical."""
    idx = np.concatenate([r[0] for r in res])
    ohard = np.concatenate([r[2] for r in res])
    oiters = np.concatenate([r[3] for r in res])
    same = np.all(hard[idx] == ohard, axis=1) & (iters[idx] == oiters)
    return {"frames": int(len(idx)), "identical": int(same.sum()), "fraction": round(float(same.mean()), 4)}


def traffic_profile(prec):
    """Committed FETCH_SIZE / WRITE_SIZE record of the headline workload's fused
    pass at storage type prec."""
    return os.path.join(ROOT, "profiles", f"k_fused_gf64_n1000_{prec}_traffic.json")


# The sources the fused pass is compiled from (its device code, the launcher
# and the compiler flags); committed counters belong to one hash of these.
KERNEL_SOURCES = ("csrc/lfsp_device.h", "csrc/lfsp_kernels.h", "csrc/kernels_q.hip", "csrc/launch.h", "build.py")


def source_sha256():
    """Hash of the fused pass's sources (KERNEL_SOURCES)."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        f = os.path.join(ROOT, "paper_1008_4370_amd", rel)
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(prec):
    """HBM bytes per k_fused launch from the committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE runs (copy-calibrated), or None when there are none for prec or
    the library sources have changed since they were taken."""
    path = traffic_profile(prec)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("source_sha256") != source_sha256():
        return None
    return t


BYTES_FORMULA = ("B = (2E+N)*q*s + 4*N*m per frame-round (read the other-check and own messages, write the new "
                 "state, read the LLRs) for each of a frame's iters rounds, plus E*q*s + 4*N*m for its first pass "
                 "(round 0 -> 1 writes the state, reads the LLRs)")


def alg_bytes(code, iters, s, first_pass=True):
    """Algorithmic HBM bytes of all fused-pass launches for one decode."""
    E, N, q, m = code.E, code.N, code.q, code.m
    per_round = (2 * E + N) * q * s + 4 * N * m
    first = E * q * s + 4 * N * m if first_pass else 0
    return int(len(iters) * first + int(np.sum(iters)) * per_round)


def time_leg(batch, llr, prec, mode, steps, max_iter, precise=None, lane_entries=None):
    """Another decoder over the same resident batch (its own code object, the
    autotuned launch choices of that storage type, optionally another
    variable-node form): Mbit/s, FER, mean rounds and the roofline fraction of
    its per-round kernels under its own storage bytes (FUSED: the fused pass;
    PLAIN: check plus variable kernels, each moving 2 E q 4 bytes per
    frame-round)."""
    import torch
    from paper_1008_4370_amd import autotune
    from paper_1008_4370_amd import decoder as D
    F = batch.llr.shape[0]
    code = D.Code.from_synth(batch.code)
    if mode == "fused":
        autotune.apply(code, prec, F)
    if precise is not None:
        code.set_tuning(precise=precise)
    if lane_entries:
        code.set_tuning(lane_entries=lane_entries)
    dec = D.Decoder(code, F, prec, mode)
    dec(llr, max_iter)
    torch.cuda.synchronize()
    # wall-clock time as the decoder runs (graph replay), then the same
    # decodes again with HIP events around every launch for the kernel time
    t0 = time.perf_counter()
    for _ in range(steps):
        out = dec(llr, max_iter)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    for k in (D.K_FUSED, D.K_CHECK, D.K_VAR):
        D.profile_read(k)
    D.profile_enable(True)
    for _ in range(steps):
        dec(llr, max_iter)
    torch.cuda.synchronize()
    D.profile_enable(False)
    kf, _ = D.profile_read(D.K_FUSED)
    kc, _ = D.profile_read(D.K_CHECK)
    kv, _ = D.profile_read(D.K_VAR)
    hard = out["hard"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    s = 4 if prec == "fp32" else 2
    if mode == "fused":
        kms = kf
        nbytes = alg_bytes(batch.code, iters, s) * steps
    else:
        kms = kc + kv
        nbytes = int(np.sum(iters)) * 4 * batch.code.E * batch.code.q * 4 * steps
    form = code.get_tuning()["precise"]
    code.close()
    leg = {"storage": prec, "mode": mode, "precise": form, "ms_per_step": round(ms, 4),
           "value": round(F * batch.info_bits_per_frame / (ms / 1e3) / 1e6, 3),
           "fer": float(np.any(hard != batch.cw, axis=1).mean()), "mean_iters": float(iters.mean()),
           "kernel_ms_per_step": round(kms / steps, 4),
           "roofline_frac": round(nbytes / (kms / 1e3) / 1e9 / HBM_PEAK_GBS, 4) if kms > 0 else None}
    return leg, hard, iters


C4_MIX = ("gf16_n2048", "gf64_n512", "gf256_n256_k16")
C5_LOADS = (20000, 50000, 100000, 150000, 200000)


def run_mixed(args):
    """Uneven multi-code batch: 3000 GF(16) N=2048, 6000 GF(64) N=512 and 2000
    GF(256) k=16 N=256 frames at 2.5 dB decoded together (one graph replay per
    chunk of passes runs all three codes on concurrent streams), against the
    same three batches decoded one after the other."""
    import torch
    from paper_1008_4370_amd import autotune, serving, synth
    from paper_1008_4370_amd import decoder as D
    batches = [synth.make_batch(w) for w in C4_MIX]
    codes = [D.Code.from_synth(b.code) for b in batches]
    tuned = [autotune.apply(c, args.prec, b.llr.shape[0]) is not None for c, b in zip(codes, batches)]
    llrs = [torch.from_numpy(b.llr).cuda() for b in batches]
    pool = D.Pool(codes, [b.llr.shape[0] for b in batches], prec=args.prec)
    # Timed three ways: steps of --chunk passes (default 8) with every code's
    # passes concurrent and a read of the active counts between steps (the
    # line's value); one step of max_iter + 1 passes (one graph launch, no host
    # read); steps of --chunk passes with the staggered schedule (the heaviest
    # code starts after the others' first --lead passes of each step, at most
    # half of the step).  The pool delivers its results to host memory
    # (harvest), so the sequential decodes below copy theirs there too.
    chunk = args.chunk or 8
    ms_form = {}
    for form, sched, lead, pps in (("chunked", 0, 0, chunk), ("one_graph", 0, 0, None),
                                   ("staggered", 1, min(args.lead, max(chunk // 2, 1)), chunk)):
        pool.set_schedule(sched, lead)
        for _ in range(args.warmup):
            serving.decode_mixed(pool, llrs, args.max_iter, pps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            r = serving.decode_mixed(pool, llrs, args.max_iter, pps)
        torch.cuda.synchronize()
        ms_form[form] = (time.perf_counter() - t0) / args.steps * 1e3
        if form == "chunked":
            res = r
    ms_mix = ms_form["chunked"]
    pool.close()
    # the same batches, one code after the other, results copied to host memory
    decs = [D.Decoder(c, b.llr.shape[0], args.prec, "fused") for c, b in zip(codes, batches)]

    def sequential():
        for d, l in zip(decs, llrs):
            o = d(l, args.max_iter)
            for key in ("hard", "iters", "status"):
                o[key].cpu()

    sequential()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sequential()
    torch.cuda.synchronize()
    ms_seq = (time.perf_counter() - t0) / args.steps * 1e3
    bits = sum(b.llr.shape[0] * b.info_bits_per_frame for b in batches)
    per_code = []
    for b, r, t in zip(batches, res, tuned):
        per_code.append({"code": f"GF({b.code.q}) k={int(round(2 * b.code.N / b.code.M))} N={b.code.N}",
                         "frames": int(b.llr.shape[0]), "fer": float(np.any(r["hard"] != b.cw, axis=1).mean()),
                         "mean_iters": float(r["iters"].mean()), "autotuned": t})
    line = {
        "metric": "decoded Mbit/s, uneven multi-code batch (3 codes, 11000 frames)",
        "value": round(bits / (ms_mix / 1e3) / 1e6, 3), "unit": "Mbit/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_mix, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3000 x GF(16)(2,4) N=2048 + 6000 x GF(64)(2,6) N=512 + 2000 x GF(256)(2,16) "
                               f"N=256, 2.5 dB, max {args.max_iter} rounds, one pool, "
                               + f"steps of {chunk} passes (one graph launch each, every code's passes "
                               "concurrent) with a read of the active counts between steps",
                   "storage": args.prec, "parallelism": "1 GPU"},
        "one_graph": {"ms_per_step": round(ms_form["one_graph"], 4),
                      "mbps": round(bits / (ms_form["one_graph"] / 1e3) / 1e6, 3)},
        "staggered": {"lead_passes": min(args.lead, max(chunk // 2, 1)), "ms_per_step": round(ms_form["staggered"], 4),
                      "mbps": round(bits / (ms_form["staggered"] / 1e3) / 1e6, 3)},
        "sequential_ms_per_step": round(ms_seq, 4),
        "sequential_mbps": round(bits / (ms_seq / 1e3) / 1e6, 3),
        "per_code": per_code, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def run_serving(args):
    """Poisson-arriving requests (32 frames, one of the three mixed-batch codes
    each, Eb/N0 uniform over 2.0..3.5 dB) at several offered loads."""
    from paper_1008_4370_amd import serving, synth
    specs = []
    for w in C4_MIX:
        d = synth.WORKLOADS[w]
        specs.append((d["m"], d["k"], d["N"]))
    banks = serving.make_banks(specs, snr_range=(2.0, 3.5), snr_points=16, frames_per_point=256)
    prec = args.prec
    sweep = []
    for load in C5_LOADS:
        r = serving.serve(banks, load, args.serve_seconds, prec=prec, max_iter=args.max_iter, request_frames=32,
                          hbm_budget=8 << 30)
        print(f"[bench] offered {load} frames/s: achieved {r['achieved_fps']:.0f}, "
              f"p50 {r['frame_latency_ms']['p50']:.2f} ms p99 {r['frame_latency_ms']['p99']:.2f} ms",
              file=sys.stderr, flush=True)
        sweep.append({k: r[k] for k in ("offered_fps", "achieved_fps", "info_mbps", "frame_latency_ms",
                                        "request_latency_ms", "frames", "fer", "slots")})
    best = max(sweep, key=lambda x: x["info_mbps"])
    line = {
        "metric": "serving Mbit/s and p50/p99 frame latency vs offered load (3 codes, Poisson arrivals)",
        "value": round(best["info_mbps"], 3), "unit": "Mbit/s", "n_gpus": 1, "steps": len(sweep), "warmup": 0,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "requests of 32 frames, uniform over GF(16)(2,4) N=2048, GF(64)(2,6) N=512, "
                               "GF(256)(2,16) N=256; Eb/N0 per request uniform over 16 points in [2.0, 3.5] dB; "
                               f"max {args.max_iter} rounds; 8 GiB of frame slots",
                   "storage": prec, "seconds_per_load": args.serve_seconds, "parallelism": "1 GPU"},
        "sweep": sweep, "roofline": None, "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="gf64_n1000",
                    help="a synthetic workload name, or 'mixed' (three codes in one pool) or 'serving' "
                         "(Poisson arrivals over the three codes at several loads)")
    ap.add_argument("--point", type=int, default=None,
                    help="Eb/N0 index into the workload's list (default: its 2.5 dB point, else its first)")
    ap.add_argument("--prec", default=None, choices=["fp32", "fp16", "bf16"],
                    help="message storage (default fp16; fp32 for the mixed workload)")
    ap.add_argument("--mode", default="fused", choices=["fused", "plain"])
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames-per-worker", type=int, default=2)
    ap.add_argument("--lane-entries", type=int, default=0, help="kernel variant (4/8/16; 0 = library default)")
    ap.add_argument("--grid-blocks", type=int, default=0, help="fused-pass grid (0 = library default)")
    ap.add_argument("--chunk", type=int, default=0, help="rounds between host checks (0 = default)")
    ap.add_argument("--lead", type=int, default=16,
                    help="mixed workload: passes of the lighter codes before the heaviest code starts")
    ap.add_argument("--no-kernel-timing", action="store_true",
                    help="skip the decodes with HIP events around every kernel launch; roofline is then omitted")
    ap.add_argument("--graphs", type=int, default=-1, help="1/0: replay captured round chunks (-1 = default)")
    ap.add_argument("--serve-load", type=float, default=100000.0,
                    help="offered frames/s of the serving phase that measures p50/p99 frame latency (0 = skip)")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--precise", action="store_true",
                    help="time the FP64 variable node (tuning key PRECISE) as the headline")
    ap.add_argument("--butterfly", action="store_true",
                    help="the FP32 butterfly variable node (tuning key PRECISE = 0; FP32 storage)")
    ap.add_argument("--decision-mfma", action="store_true",
                    help="with --butterfly: the decision's transforms as FP16 MFMAs (tuning key DECISION_MFMA = 1)")
    ap.add_argument("--no-logsp-variant", action="store_true",
                    help="skip timing the conventional log-domain SP decoder on the same batch")
    ap.add_argument("--no-precise-variant", action="store_true",
                    help="skip the extra timing of the FP64 variable node")
    ap.add_argument("--no-legs", action="store_true",
                    help="skip the other storage type's and the PLAIN FP32 decoder's timing")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a device-to-device copy of MIB MiB (calibrates rocprofv3 "
                         "FETCH_SIZE/WRITE_SIZE against a known byte count) and exit")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "frames would shard across GPUs with no per-round exchange.", file=sys.stderr)
        sys.exit(2)

    if args.prec is None:
        # 16-bit message storage (pmf words) decodes at the FP32 frame error
        # rate in fewer bytes; the uneven batch is specified with FP32 messages
        args.prec = "fp32" if args.workload == "mixed" else "fp16"
    if args.workload == "mixed":
        return run_mixed(args)
    if args.workload == "serving":
        return run_serving(args)
    from paper_1008_4370_amd import synth
    if args.point is None:
        pts = synth.WORKLOADS[args.workload]["ebn0"]
        args.point = pts.index(2.5) if 2.5 in pts else 0
    batch = synth.make_batch(args.workload, point=args.point)
    F = batch.llr.shape[0]
    cpu, cpu_res = None, None
    if not args.no_cpu_baseline:
        print("[bench] cpu_baseline: FP64 oracle on a sample ...", file=sys.stderr, flush=True)
        cpu, cpu_res = cpu_baseline(batch, args.max_iter, args.cpu_frames_per_worker)
        print(f"[bench] cpu_baseline done: {cpu['value']:.4f} Mbit/s", file=sys.stderr, flush=True)

    import torch
    from paper_1008_4370_amd import decoder as D
    code = D.Code.from_synth(batch.code)
    from paper_1008_4370_amd import autotune
    tuned = autotune.apply(code, args.prec, F) is not None
    tune = {k: v for k, v in (("lane_entries", args.lane_entries), ("grid_blocks", args.grid_blocks),
                              ("chunk", args.chunk)) if v}
    if args.graphs >= 0:
        tune["graphs"] = args.graphs
    if tune:
        code.set_tuning(**tune)
    if args.precise:
        code.set_tuning(precise=1)
    if args.butterfly or args.decision_mfma:
        code.set_tuning(precise=0, decision_mfma=int(args.decision_mfma))
    default_form = not (args.precise or args.butterfly or args.decision_mfma)
    dec = D.Decoder(code, F, args.prec, args.mode)
    llr = torch.from_numpy(batch.llr).cuda()
    for _ in range(args.warmup):
        dec(llr, args.max_iter)
    torch.cuda.synchronize()
    kernel = D.K_FUSED if args.mode == "fused" else D.K_CHECK
    # The timed steps run as the decoder runs in production (captured chunks
    # of rounds replayed as graphs, where the library uses them).
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        out = dec(llr, args.max_iter)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_step = (t1 - t0) / args.steps * 1e3
    # Kernel durations: the same steps again with a pair of HIP events on the
    # decode stream around every launch of the per-round kernels (HIP cannot
    # time kernels inside a replayed graph, so these decodes launch every pass
    # from the host; the kernels and their results are the same).
    kms, launches, ms_var, ms_step_events = 0.0, 0, 0.0, None
    if not args.no_kernel_timing:
        D.profile_read(D.K_FUSED), D.profile_read(D.K_CHECK), D.profile_read(D.K_VAR)
        D.profile_enable(True)
        te0 = time.perf_counter()
        for _ in range(args.steps):
            dec(llr, args.max_iter)
        torch.cuda.synchronize()
        ms_step_events = (time.perf_counter() - te0) / args.steps * 1e3
        D.profile_enable(False)
        kms, launches = D.profile_read(kernel)
        ms_var, _ = D.profile_read(D.K_VAR)

    precise_line = prob_line = None
    if args.mode == "fused" and default_form and not args.no_precise_variant:
        # The same batch with the other FP32 variable-node forms (FP32 storage;
        # 16-bit pmf words are read by the default form only): the FP64
        # variable node (tuning key PRECISE = 1, 8 entries per lane where the
        # code has that variant) and the FP32 butterfly form (PRECISE = 0).
        lane = 8 if code.kmax <= 8 and code.m >= 3 else None
        precise_line, _, _ = time_leg(batch, llr, "fp32", "fused", args.steps, args.max_iter, precise=1,
                                      lane_entries=lane)
        prob_line, _, _ = time_leg(batch, llr, "fp32", "fused", args.steps, args.max_iter, precise=0)

    logsp_line = None
    if args.mode == "fused" and not args.no_logsp_variant:
        # The same batch through the conventional log-domain SP decoder (the
        # comparison of Table 1): whole-decode time, and the time of its check
        # and variable kernels per frame-round next to the fused pass's.
        def logsp_leg(prec):
            ldec = D.Decoder(code, F, prec, "logsp")
            ldec(llr, args.max_iter)
            torch.cuda.synchronize()
            tl0 = time.perf_counter()
            for _ in range(args.steps):
                lout = ldec(llr, args.max_iter)
            torch.cuda.synchronize()
            lms = (time.perf_counter() - tl0) / args.steps * 1e3
            # kernel times from further decodes with HIP events per launch
            D.profile_read(D.K_CHECK), D.profile_read(D.K_VAR)
            D.profile_enable(not args.no_kernel_timing)
            for _ in range(args.steps):
                ldec(llr, args.max_iter)
            torch.cuda.synchronize()
            D.profile_enable(False)
            ck, _ = D.profile_read(D.K_CHECK)
            vk, _ = D.profile_read(D.K_VAR)
            lhard = lout["hard"].cpu().numpy()
            lrounds = int(lout["iters"].sum())
            del ldec
            return {"ms_per_step": round(lms, 4),
                    "value": round(F * batch.info_bits_per_frame / (lms / 1e3) / 1e6, 3),
                    "fer": float(np.any(lhard != batch.cw, axis=1).mean()),
                    "mean_iters": float(lout["iters"].float().mean()),
                    "check_kernel_ms_per_step": round(ck / args.steps, 4),
                    "var_kernel_ms_per_step": round(vk / args.steps, 4),
                    "ns_per_frame_round": round((ck + vk) / args.steps * 1e6 / max(lrounds, 1), 2)}

        logsp_line = logsp_leg("fp32")
        logsp_line["lfsp_ns_per_frame_round"] = round(kms / args.steps * 1e6 / max(int(out["iters"].sum()), 1), 2)
        logsp_line["lfsp_speedup"] = round(logsp_line["ms_per_step"] / ms_step, 3)
        # The same decoder with one byte per message entry (log2 probabilities
        # on the integer grid, the 8-bit message memory of the quantisation
        # argument): a quarter of the message traffic.
        logsp_line["log8"] = logsp_leg("log8")

    legs = None
    if args.mode == "fused" and default_form and not args.no_legs:
        # The comparison the precision plan sets: the 16-bit-storage decoder
        # against the FP32 decoders on the same frames (the other storage type
        # of the fused decoder, and the PLAIN two-kernel FP32 decoder).
        legs = {}
        other = "fp16" if args.prec == "fp32" else "fp32"
        legs[other], lh, li = time_leg(batch, llr, other, "fused", args.steps, args.max_iter)
        if cpu_res is not None:
            legs[other]["oracle_agreement"] = oracle_agreement(cpu_res, lh, li)
        legs["plain_fp32"], lh, li = time_leg(batch, llr, "fp32", "plain", args.steps, args.max_iter)
        if cpu_res is not None:
            legs["plain_fp32"]["oracle_agreement"] = oracle_agreement(cpu_res, lh, li)
        print(f"[bench] legs: " + ", ".join(f"{k} {v['value']:.1f} Mbit/s FER {v['fer']:.2e}"
                                             for k, v in legs.items()), file=sys.stderr, flush=True)

    serve = None
    if args.serve_load > 0:
        # Continuous batching of the same frames arriving as a Poisson process
        # (requests of 32 frames), same storage precision; latency is arrival
        # to harvest on the host.
        from paper_1008_4370_amd import serving
        bank = serving.bank_from_batch(batch, code)
        budget = 1024 * serving.D.pool_slot_bytes(code, args.prec)   # 1024 frame slots
        serve = serving.serve([bank], args.serve_load, args.serve_seconds, prec=args.prec, max_iter=args.max_iter,
                              request_frames=32, hbm_budget=budget, warmup_s=0.5)
        print(f"[bench] serving at {args.serve_load:.0f} frames/s: {serve['achieved_fps']:.0f} frames/s, "
              f"p50 {serve['frame_latency_ms']['p50']:.2f} ms, p99 {serve['frame_latency_ms']['p99']:.2f} ms",
              file=sys.stderr, flush=True)

    hard = out["hard"].cpu().numpy()
    iters = out["iters"].cpu().numpy()
    status = out["status"].cpu().numpy()
    info_bits = batch.info_bits_per_frame
    value = F * info_bits / (ms_step / 1e3) / 1e6
    frame_err = np.any(hard != batch.cw, axis=1)
    bit_err = int(np.sum((((hard.astype(np.int64) ^ batch.cw)[..., None] >> np.arange(batch.code.m)) & 1)))
    s = 4 if args.prec == "fp32" else 2
    achieved_rounds = None
    if kms <= 0:
        achieved, roof_kernel = None, None
    elif args.mode == "fused":
        total_bytes = alg_bytes(batch.code, iters, s) * args.steps
        achieved = total_bytes / (kms / 1e3) / 1e9
        # the same kernel time over iters x B alone (first passes not counted)
        achieved_rounds = alg_bytes(batch.code, iters, s, first_pass=False) * args.steps / (kms / 1e3) / 1e9
        roof_kernel = "k_fused"
    else:
        # PLAIN: check + variable kernels each move 2*E*q*4 bytes per frame-round
        E, q = batch.code.E, batch.code.q
        total_bytes = int(np.sum(iters)) * 4 * E * q * 4 * args.steps
        achieved = total_bytes / ((kms + ms_var) / 1e3) / 1e9
        roof_kernel = "k_check_plain+k_var_plain"
    # measured HBM bytes per k_fused launch (committed counters) for this exact
    # configuration: default workload, FP32 storage, fused, tuned defaults
    traffic, traffic_note = None, "no counters for this configuration"
    if (args.workload == "gf64_n1000" and args.mode == "fused" and default_form
            and not tune and args.point == 2 and args.max_iter == 100):
        t = measured_traffic(args.prec)
        if t is None:
            traffic_note = "no counters for the current kernel sources"
        else:
            traffic = int(round(t["traffic_bytes_per_launch"]))
            traffic_note = (f"HBM bytes per launch from FETCH_SIZE x {t['fetch_factor']:.3f} + WRITE_SIZE x "
                            f"{t['write_factor']:.3f} (KiB, copy-calibrated), mean of {t['launches']} launches of one "
                            f"decode; algorithmic {int(round(t['alg_bytes_per_launch']))} bytes per launch")
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: GF({batch.code.q}) (2,{int(round(2 * batch.code.N / batch.code.M))}) "
                        f"N={batch.code.N} M={batch.code.M}, {F} frames, Eb/N0={batch.ebn0} dB, "
                        f"max {args.max_iter} rounds",
            "storage": args.prec,
            "mode": args.mode,
            "frames": F,
            "info_bits_per_frame": info_bits,
            "parallelism": "1 GPU",
            "tuning": code.get_tuning(),
            "autotuned": tuned and not tune,
        },
        "roofline": None if achieved is None else {
            "traffic": traffic,
            "traffic_note": traffic_note,
            "bound": "hbm",
            "kernel": roof_kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "bytes": BYTES_FORMULA if args.mode == "fused" else "4*E*q*4 per frame-round (check + variable kernels)",
            "frac_rounds_only": None if achieved_rounds is None else round(achieved_rounds / HBM_PEAK_GBS, 4),
            "launches": int(launches),
            "kernel_ms_per_step": round(kms / args.steps, 4),
            "timing": f"HIP events around every launch over {args.steps} further decodes of the same batch "
                      f"(eager launches: {ms_step_events:.3f} ms per decode)" if ms_step_events else None,
        },
        "cpu_baseline": None if cpu is None else dict(cpu, agreement=oracle_agreement(cpu_res, hard, iters)),
        "legs": legs,
        "precise_variant": precise_line,
        "butterfly_variant": prob_line,
        "logsp_variant": logsp_line,
        "fer": float(frame_err.mean()),
        "ber": bit_err / (F * batch.code.N * batch.code.m),
        "mean_iters": float(iters.mean()),
        "max_iters": int(iters.max()),
        "converged": float(((status & 1) != 0).mean()),
        "latency_ms": None if serve is None else {
            "p50": round(serve["frame_latency_ms"]["p50"], 3),
            "p99": round(serve["frame_latency_ms"]["p99"], 3),
            "request_p50": round(serve["request_latency_ms"]["p50"], 3),
            "request_p99": round(serve["request_latency_ms"]["p99"], 3),
            "offered_fps": args.serve_load,
            "achieved_fps": round(serve["achieved_fps"], 1),
            "serving_mbps": round(serve["info_mbps"], 3),
            "slots": serve["slots"][0],
            "note": "frame arrival (Poisson, requests of 32 frames) to harvest, continuous batching",
        },
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
