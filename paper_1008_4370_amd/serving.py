"""Serving loop over the decoding pool (continuous batching).

Requests arrive as a Poisson process in wall-clock time; each request carries
`request_frames` frames of one code (chosen uniformly) at one Eb/N0 (uniform
over the given range).  Requests are admitted FIFO per code into free frame
slots, whose number per code follows from an HBM budget: an equal share per
code and the most slots whose device bytes fit it (ldpc_fd_pool_budget_slots).  Between admissions the pool
runs a chunk of passes over every active frame of every code; stopped frames
are harvested and their slots freed at once, so new requests join frames in
flight.  Reported: per-frame and per-request latency (arrival to harvest)
percentiles, decoded information Mbit/s, FER per code.

Channel frames are drawn from a device-resident bank generated beforehand
(random codewords of each code over BPSK/AWGN at `snr_points` Eb/N0 values
spread uniformly over the range), so the loop measures decoding, not noise
generation.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass

import numpy as np

from . import decoder as D
from . import synth


@dataclass
class CodeBank:
    code: synth.Code
    enc: synth.Encoder
    gcode: D.Code
    ebn0: np.ndarray        # [P]
    cw: np.ndarray          # [P, B, N] transmitted codewords (host, for FER)
    llr: object             # torch [P, B, N, m] on the device


def make_banks(specs, snr_range=(2.0, 3.5), snr_points=16, frames_per_point=256, seed=2024, device="cuda"):
    """specs: list of (m, k, N).  Returns one CodeBank per code."""
    import torch
    banks = []
    pts = np.linspace(snr_range[0], snr_range[1], snr_points)
    for i, (m, k, N) in enumerate(specs):
        code = synth.make_code(N, k, m, seed_graph=seed + 10 * i + 1, seed_labels=seed + 10 * i + 2)
        enc = synth.Encoder(code)
        cws, llrs = [], []
        for p, e in enumerate(pts):
            cw = synth.random_codewords(enc, frames_per_point, seed=seed + 1000 * i + 2 * p + 3)
            llr = synth.bpsk_awgn_llr(cw, m, e, code.design_rate, seed=seed + 1000 * i + 2 * p + 4)
            cws.append(cw)
            llrs.append(llr)
        banks.append(CodeBank(code, enc, D.Code.from_synth(code), pts,
                              np.stack(cws), torch.from_numpy(np.stack(llrs)).to(device)))
    return banks


def bank_from_batch(batch, gcode=None, device="cuda"):
    """A one-point bank over the frames of a synth.Batch (one code, one Eb/N0)."""
    import torch
    gcode = gcode or D.Code.from_synth(batch.code)
    return CodeBank(batch.code, batch.enc, gcode, np.array([batch.ebn0]), batch.cw[None],
                    torch.from_numpy(batch.llr[None]).to(device))


def slots_for_budget(banks, hbm_budget: int, prec: str):
    """The slot counts of a pool sized from the budget: an equal share per
    code, the most slots whose device bytes fit it."""
    return D.pool_budget_slots([b.gcode for b in banks], hbm_budget, prec)


def serve(banks, offered_fps: float, duration_s: float, prec: str = "fp16", max_iter: int = 100,
          request_frames: int = 32, hbm_budget: int = 8 << 30, passes_per_step: int = 2, seed: int = 7,
          warmup_s: float = 0.5, record: bool = False):
    """Run the serving loop for `duration_s` seconds of arrivals (after a warm-up).

    Requests live in arrays indexed by request id; a harvest's frames are
    booked with array operations (no per-frame Python work between steps).
    With `record`, the result also lists (code, Eb/N0 index, bank frame,
    iterations, hard decision) for every returned frame."""
    rng = np.random.default_rng(seed)
    # each code's autotuned launch choices for a batch of its slot count (the
    # pool captures its steps with the codes' tuning at that time)
    from . import autotune
    for b, n in zip(banks, slots_for_budget(banks, hbm_budget, prec)):
        autotune.apply(b.gcode, prec, n)
    pool = D.Pool([b.gcode for b in banks], None, prec=prec, hbm_budget=hbm_budget)
    slots = pool.slots
    ncodes = len(banks)
    B = banks[0].llr.shape[1]
    req_rate = offered_fps / request_frames
    cap = int(req_rate * (warmup_s + duration_s) * 1.5) + 1024
    r_code = np.zeros(cap, np.int64)
    r_point = np.zeros(cap, np.int64)
    r_first = np.zeros(cap, np.int64)
    r_arr = np.zeros(cap, np.float64)
    r_admitted = np.zeros(cap, np.int64)
    r_done = np.zeros(cap, np.int64)
    r_tdone = np.full(cap, np.nan)
    queues = [collections.deque() for _ in range(ncodes)]
    tag_base = 1 << 20                # tag = rid * tag_base + frame index
    lat_arr, lat_val = [], []         # per harvest: arrival times and latencies (arrays)
    info_bits = 0
    frame_err = [0] * ncodes
    frames_done = [0] * ncodes
    records = []
    t0 = time.perf_counter()
    next_arr = t0 + warmup_s + rng.exponential(1.0 / req_rate)
    t_end = t0 + warmup_s + duration_s
    nreq = 0
    open_reqs = 0
    measure_start = t0 + warmup_s
    steps = 0
    bits_per_frame = [b.enc.K * b.code.m for b in banks]
    while True:
        now = time.perf_counter()
        while next_arr <= now and next_arr < t_end:
            if nreq == cap:
                raise RuntimeError("request table full")
            k = int(rng.integers(ncodes))
            r_code[nreq], r_point[nreq] = k, int(rng.integers(len(banks[k].ebn0)))
            r_first[nreq], r_arr[nreq] = int(rng.integers(0, B - request_frames + 1)), next_arr
            queues[k].append(nreq)
            nreq += 1
            open_reqs += 1
            next_arr += rng.exponential(1.0 / req_rate)
        # admission (FIFO per code, partial admission allowed)
        for k in range(ncodes):
            while queues[k]:
                rid = queues[k][0]
                lo = int(r_first[rid] + r_admitted[rid])
                cnt = request_frames - int(r_admitted[rid])
                tags = rid * tag_base + np.arange(r_admitted[rid], request_frames)
                got = pool.submit(k, banks[k].llr[r_point[rid], lo:lo + cnt], tags, max_iter)
                r_admitted[rid] += got
                if r_admitted[rid] < request_frames:
                    break
                queues[k].popleft()
        pool.step(passes_per_step)
        steps += 1
        now = time.perf_counter()
        for k in range(ncodes):
            tags, it, st, hd = pool.harvest(k, slots[k])
            n = len(tags)
            if n == 0:
                continue
            t_h = time.perf_counter()
            rids = (tags // tag_base).astype(np.int64)
            fis = (tags % tag_base).astype(np.int64)
            arr = r_arr[rids]
            lat_arr.append(arr)
            lat_val.append(t_h - arr)
            frames_done[k] += n
            sent = banks[k].cw[r_point[rids], r_first[rids] + fis]
            frame_err[k] += int(np.any(hd != sent, axis=1).sum())
            info_bits += int((arr >= measure_start).sum()) * bits_per_frame[k]
            if record:
                records.extend((k, int(r_point[r]), int(r_first[r] + f), int(i), h.copy())
                               for r, f, i, h in zip(rids, fis, it, hd))
            np.add.at(r_done, rids, 1)
            fin = np.unique(rids[r_done[rids] == request_frames])
            r_tdone[fin] = t_h
            open_reqs -= len(fin)
        if now >= t_end and open_reqs == 0:
            break
        if now >= t_end + 30.0:
            raise RuntimeError("serving loop did not drain within 30 s after the last arrival")
    t_last = time.perf_counter()
    pool.close()
    la = np.concatenate(lat_arr) if lat_arr else np.zeros(0)
    lv = np.concatenate(lat_val) if lat_val else np.zeros(0)
    fl = lv[la >= measure_start] * 1e3
    meas = (r_arr[:nreq] >= measure_start) & np.isfinite(r_tdone[:nreq])
    rl = (r_tdone[:nreq] - r_arr[:nreq])[meas] * 1e3
    elapsed = t_last - measure_start
    out = {
        "offered_fps": offered_fps,
        "achieved_fps": float(len(fl) / elapsed) if elapsed > 0 else 0.0,
        "info_mbps": info_bits / elapsed / 1e6 if elapsed > 0 else 0.0,
        "frame_latency_ms": {"p50": float(np.percentile(fl, 50)) if len(fl) else None,
                             "p99": float(np.percentile(fl, 99)) if len(fl) else None},
        "request_latency_ms": {"p50": float(np.percentile(rl, 50)) if len(rl) else None,
                               "p99": float(np.percentile(rl, 99)) if len(rl) else None},
        "frames": int(len(fl)),
        "fer": [frame_err[k] / max(frames_done[k], 1) for k in range(ncodes)],
        "slots": slots,
        "steps": steps,
        "prec": prec,
    }
    if record:
        out["records"] = records
    return out


def decode_mixed(pool: D.Pool, llrs, max_iter: int = 100, passes_per_step: int | None = 8):
    """Decode one batch per pool code together: every frame is admitted at
    once (the pool needs as many slots as frames).  Steps of passes_per_step
    passes (each one graph launch running every pass of every code with active
    frames on concurrent streams) alternate with reads of the codes' active
    counts, from which the next step picks each code's kernel forms (the
    few-frames forms once a code's active count is within its tail threshold)
    and leaves out codes with no active frame; a code is harvested as soon as
    none of its frames is active.  passes_per_step=None: one step of
    max_iter + 1 passes (a frame needs at most that many) with no host read in
    between, then every code is harvested.  Returns, per code, dict(iters,
    status, hard) in frame order."""
    ncodes = len(llrs)
    for k, llr in enumerate(llrs):
        F = int(llr.shape[0])
        got = pool.submit(k, llr, np.arange(F, dtype=np.uint64), max_iter)
        if got != F:
            raise ValueError(f"pool code {k}: {F} frames but only {got} free slots")
    got = [None] * ncodes

    def harvest(k):
        F = int(llrs[k].shape[0])
        tags, it, st, hd = pool.harvest(k, F)
        if len(tags) != F:
            raise RuntimeError(f"pool code {k}: harvested {len(tags)} of {F} frames")
        order = np.argsort(tags)
        got[k] = {"iters": it[order], "status": st[order], "hard": hd[order]}

    if passes_per_step is None:
        pool.step(max_iter + 1)
        for k in range(ncodes):
            harvest(k)
        return got
    passes = 0
    while passes < max_iter + 1:
        n = min(passes_per_step, max_iter + 1 - passes)
        pool.step(n)
        passes += n
        for k in range(ncodes):
            if got[k] is None and pool.active(k) == 0:
                harvest(k)
        if all(g is not None for g in got):
            return got
    raise RuntimeError("frames still active after max_iter + 1 passes")
