"""Autotuner for the fused decoder's launch choices.

For one code and storage precision it times complete decodes of a synthetic
batch (random codewords of the code over BPSK/AWGN) for every combination of
  - entries per lane (4, 8, 16: the kernel variant; each lane holds R entries
    of a frame's q-point vectors, a wave holds 64 / (q / R) frames),
  - grid blocks of the fused pass (workgroups of 256 threads, a multiple of 8
    so that every XCD gets the same share),
  - rounds per host check (graph chunk),
  - the variant used once few frames are left and its threshold,
keeps the fastest, and stores it in a JSON table keyed by
(m, kmax, N, E, precision, frames bucket).  `apply(code, prec, frames)` sets a
code's tuning from the table (library defaults when the key is absent).
"""
from __future__ import annotations

import itertools
import json
import os
import time

from . import decoder as D
from . import synth

TABLE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")


def frames_bucket(F: int) -> int:
    """Power-of-two bucket of a batch size (tuning depends on it only coarsely)."""
    return 1 << max(0, int(F - 1).bit_length())


def key(code: D.Code, prec: str, frames: int) -> str:
    m, kmax, N, E = code.m, code.kmax, code.N, code.E
    return f"m{m}_k{kmax}_N{N}_E{E}_{prec}_F{frames_bucket(frames)}"


def lane_choices(m: int, kmax: int):
    q = 1 << m
    out = [4]
    if kmax <= 16 and q >= 8:
        out.append(8)
    if kmax <= 8 and q >= 16:
        out.append(16)
    return out


def load_table(path: str = TABLE) -> dict:
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def apply(code: D.Code, prec: str, frames: int, path: str = TABLE) -> dict | None:
    """Set the tuned launch choices on `code`; returns them (None if untuned)."""
    ent = load_table(path).get(key(code, prec, frames))
    if ent is None:
        return None
    code.set_tuning(lane_entries=ent["lane_entries"], grid_blocks=ent["grid_blocks"], chunk=ent["chunk"],
                    graphs=1)
    if "tail_entries" in ent:
        code.set_tuning(tail_entries=ent["tail_entries"], tail_frames=ent["tail_frames"])
    code.set_tuning(tail_chunk=ent.get("tail_chunk", 0), batch_retire=ent.get("batch_retire", 0),
                    first_chunk=ent.get("first_chunk", 0))
    return ent


def _time_decode(dec, llr, max_iter, reps):
    import torch
    dec(llr, max_iter)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        t0 = time.perf_counter()
        dec(llr, max_iter)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    return best


def tune(code: D.Code, llr, prec: str = "fp32", max_iter: int = 100, reps: int = 3,
         grid_blocks=(2048, 4096, 8192, 16384, 32768), chunks=(4, 8), tail_frames=(0, 32, 128, 512, 2048, 1 << 20),
         tail_chunks=(0, 16, 32), later_chunks=(2, 3), path: str | None = TABLE, log=None) -> dict:
    """Sweep the launch choices for decoding `llr` (device [F][N][m]) and record
    the best: first the main variant, grid and chunk (tail variant at its
    defaults), then the tail variant and its threshold, then the number of
    passes per captured graph in the tail, then batched retirement of the tail
    (with the tail chunk chosen again), then shorter chunks after a first chunk
    of the chosen length."""
    m, kmax, N = code.m, code.kmax, code.N
    F = int(llr.shape[0])
    dec = D.Decoder(code, F, prec, "fused")
    default = code.get_tuning()
    default_ms = _time_decode(dec, llr, max_iter, reps) * 1e3

    def run(**kw):
        code.set_tuning(graphs=1, **{"tail_chunk": 0, "batch_retire": 0, "first_chunk": 0, **kw})
        t = _time_decode(dec, llr, max_iter, reps)
        if log:
            log(f"[autotune] m={m} k={kmax} N={N} {prec} F={F}: {kw}: {t * 1e3:.3f} ms")
        return t

    main = []
    for le, gb, ch in itertools.product(lane_choices(m, kmax), grid_blocks, chunks):
        main.append((run(lane_entries=le, grid_blocks=gb, chunk=ch, tail_entries=default["tail_entries"],
                         tail_frames=default["tail_frames"]), le, gb, ch))
    t_main, le, gb, ch = min(main)
    tail = [(t_main, default["tail_entries"], default["tail_frames"])]
    for te, tf in itertools.product(lane_choices(m, kmax), tail_frames):
        tail.append((run(lane_entries=le, grid_blocks=gb, chunk=ch, tail_entries=te, tail_frames=tf), te, tf))
    t, te, tf = min(tail)
    base = dict(lane_entries=le, grid_blocks=gb, chunk=ch, tail_entries=te, tail_frames=tf)
    tcs = [(t, 0)]
    for tc in tail_chunks:
        if tc:
            tcs.append((run(**base, tail_chunk=tc), tc))
    t, tc = min(tcs)
    brs = [(t, 0, tc)]
    for tcb in tail_chunks:
        brs.append((run(**base, tail_chunk=tcb, batch_retire=1), 1, tcb))
    t, br, tc = min(brs)
    fcs = [(t, 0, ch)]
    for later in later_chunks:
        if later < ch:
            fcs.append((run(**{**base, "chunk": later}, tail_chunk=tc, batch_retire=br, first_chunk=ch), ch, later))
    t, fc, ch_after = min(fcs)
    ent = {"lane_entries": le, "grid_blocks": gb, "chunk": ch_after, "first_chunk": fc, "tail_entries": te,
           "tail_frames": tf, "tail_chunk": tc, "batch_retire": br, "ms": round(t * 1e3, 4),
           "default_ms": round(default_ms, 4),
           "default": {k: default[k] for k in ("lane_entries", "grid_blocks", "chunk", "tail_entries",
                                               "tail_frames")},
           "swept": len(main) + len(tail) + len(tcs) + len(brs) + len(fcs) - 4}
    code.set_tuning(lane_entries=le, grid_blocks=gb, chunk=ch_after, first_chunk=fc, tail_entries=te,
                    tail_frames=tf, tail_chunk=tc, batch_retire=br, graphs=1)
    if path:
        table = load_table(path)
        table[key(code, prec, F)] = ent
        with open(path, "w") as fh:
            json.dump(table, fh, indent=1, sort_keys=True)
    return ent


def tune_workload(name: str, prec: str = "fp32", frames: int | None = None, point: int | None = None,
                  max_iter: int = 100, path: str | None = TABLE, log=print) -> dict:
    """Tune on a named synthetic workload (synth.WORKLOADS)."""
    import torch
    if point is None:
        pts = synth.WORKLOADS[name]["ebn0"]
        point = pts.index(2.5) if 2.5 in pts else 0
    b = synth.make_batch(name, frames=frames, point=point)
    code = D.Code.from_synth(b.code)
    ent = tune(code, torch.from_numpy(b.llr).cuda(), prec, max_iter, path=path, log=log)
    code.close()
    return ent


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="tune the fused decoder's launch choices on synthetic workloads")
    ap.add_argument("workloads", nargs="+")
    ap.add_argument("--prec", default="fp32")
    ap.add_argument("--frames", type=int, default=None)
    ap.add_argument("--point", type=int, default=None)
    ap.add_argument("--table", default=TABLE)
    a = ap.parse_args()
    for w in a.workloads:
        print(json.dumps({w: tune_workload(w, a.prec, a.frames, a.point, path=a.table)}), flush=True)
