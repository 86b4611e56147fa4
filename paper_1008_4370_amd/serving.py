"""Serving loop over the decoding pool (continuous batching).

Requests arrive as a Poisson process in wall-clock time; each request carries
`request_frames` frames of one code (chosen uniformly) at one Eb/N0 (uniform
over the given range).  Requests are admitted FIFO per code into free frame
slots, whose number per code follows from an HBM budget divided by the
per-slot footprint (ldpc_fd_pool_slot_bytes).  Between admissions the pool
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
from dataclasses import dataclass, field

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


@dataclass
class Request:
    rid: int
    code: int
    point: int
    first: int              # first frame in the bank bucket
    n: int
    t_arrival: float
    admitted: int = 0
    done: int = 0
    t_done: float = 0.0
    frame_done: list = field(default_factory=list)


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
    """Equal share of the budget per code, divided by the per-slot footprint."""
    share = hbm_budget // len(banks)
    return [max(1, share // D.pool_slot_bytes(b.gcode, prec)) for b in banks]


def serve(banks, offered_fps: float, duration_s: float, prec: str = "fp16", max_iter: int = 100,
          request_frames: int = 32, hbm_budget: int = 8 << 30, passes_per_step: int = 2, seed: int = 7,
          warmup_s: float = 0.5, record: bool = False):
    """Run the serving loop for `duration_s` seconds of arrivals (after a warm-up).

    With `record`, the result also lists (code, Eb/N0 index, bank frame,
    iterations, hard decision) for every returned frame."""
    rng = np.random.default_rng(seed)
    slots = slots_for_budget(banks, hbm_budget, prec)
    pool = D.Pool([b.gcode for b in banks], slots, prec=prec)
    ncodes = len(banks)
    B = banks[0].llr.shape[1]
    req_rate = offered_fps / request_frames
    queues = [collections.deque() for _ in range(ncodes)]
    reqs = {}
    tag_base = 1 << 20                # tag = rid * tag_base + frame index
    frame_lat, req_lat = [], []
    info_bits = 0
    frame_err = [0] * ncodes
    frames_done = [0] * ncodes
    records = []
    t0 = time.perf_counter()
    next_arr = t0 + warmup_s + rng.exponential(1.0 / req_rate)
    t_end = t0 + warmup_s + duration_s
    rid = 0
    measure_start = t0 + warmup_s
    steps = 0
    while True:
        now = time.perf_counter()
        while next_arr <= now and next_arr < t_end:
            k = int(rng.integers(ncodes))
            p = int(rng.integers(len(banks[k].ebn0)))
            first = int(rng.integers(0, B - request_frames + 1))
            r = Request(rid, k, p, first, request_frames, next_arr)
            reqs[rid] = r
            queues[k].append(r)
            rid += 1
            next_arr += rng.exponential(1.0 / req_rate)
        # admission (FIFO per code, partial admission allowed)
        for k in range(ncodes):
            while queues[k]:
                r = queues[k][0]
                bank = banks[k]
                lo = r.first + r.admitted
                cnt = r.n - r.admitted
                tags = r.rid * tag_base + np.arange(r.admitted, r.n)
                got = pool.submit(k, bank.llr[r.point, lo:lo + cnt], tags, max_iter)
                r.admitted += got
                if r.admitted < r.n:
                    break
                queues[k].popleft()
        pool.step(passes_per_step)
        steps += 1
        now = time.perf_counter()
        for k in range(ncodes):
            tags, it, st, hd = pool.harvest(k, slots[k])
            if len(tags) == 0:
                continue
            t_h = time.perf_counter()
            for i, t in enumerate(tags):
                r = reqs[int(t) // tag_base]
                fi = int(t) % tag_base
                r.done += 1
                frame_lat.append((r.t_arrival, t_h - r.t_arrival))
                frames_done[k] += 1
                if record:
                    records.append((k, r.point, r.first + fi, int(it[i]), hd[i].copy()))
                if not np.array_equal(hd[i], banks[k].cw[r.point, r.first + fi]):
                    frame_err[k] += 1
                if r.t_arrival >= measure_start:
                    info_bits += banks[k].enc.K * banks[k].code.m
                if r.done == r.n:
                    r.t_done = t_h
                    req_lat.append((r.t_arrival, t_h - r.t_arrival))
                    del reqs[r.rid]
        if now >= t_end and not reqs:
            break
        if now >= t_end + 30.0:
            raise RuntimeError("serving loop did not drain within 30 s after the last arrival")
    t_last = time.perf_counter()
    pool.close()
    fl = np.array([l for a, l in frame_lat if a >= measure_start]) * 1e3
    rl = np.array([l for a, l in req_lat if a >= measure_start]) * 1e3
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


def decode_mixed(pool: D.Pool, llrs, max_iter: int = 100, passes_per_step: int = 4):
    """Decode one batch per pool code together: every frame is admitted at
    once (the pool needs as many slots as frames), each step replays one graph
    that runs `passes_per_step` passes of every code on concurrent streams,
    and each code is harvested as soon as none of its frames is active (which
    leaves it out of later steps).  Returns, per code, dict(iters, status,
    hard) in frame order."""
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

    # a code whose frames have all stopped is harvested at once, which takes it
    # out of the following steps
    for _ in range((max_iter + passes_per_step) // passes_per_step + 1):
        pool.step(passes_per_step)
        for k in range(ncodes):
            if got[k] is None and pool.active(k) == 0:
                harvest(k)
        if all(g is not None for g in got):
            break
    else:
        raise RuntimeError("frames still active after max_iter + 1 passes")
    return got
