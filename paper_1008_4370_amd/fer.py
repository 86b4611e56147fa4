"""Frame-error-rate curves of the GPU decoder, for comparing storage precisions.

Each Eb/N0 point decodes batches of random codewords of the workload's code
over BPSK/AWGN until `max_errors` frame errors or `max_frames` frames.  The
codewords come from the workload's systematic encoder (a bank of `batch`
codewords drawn once); the noise of every batch is drawn on the device from a
seeded generator, so the LLR recipe is the one of synth.bpsk_awgn_llr
(LLR = 2 y / sigma^2) with a fresh noise realisation per batch.

`gap_db(a, b, fer)` reads the Eb/N0 at which each curve crosses `fer` by
linear interpolation of log10(FER) against Eb/N0 and returns b - a.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np

from . import decoder as D
from . import synth


def wilson(k: int, n: int, z: float = 1.96):
    """95% Wilson score interval of a binomial proportion k / n."""
    if n == 0:
        return (0.0, 1.0)
    p = k / n
    d = 1 + z * z / n
    c = (p + z * z / (2 * n)) / d
    h = z * math.sqrt(p * (1 - p) / n + z * z / (4 * n * n)) / d
    return (max(0.0, c - h), min(1.0, c + h))


def fer_curve(workload: str = "gf64_n1000", prec: str = "fp32", points=None, max_errors: int = 100,
              max_frames: int = 1 << 20, batch: int = 4096, max_iter: int = 100, seed: int = 77,
              precise: int | None = None, log=None, mode: str = "fused", quant_bits: int = 0,
              quant_step: int = 256) -> list[dict]:
    import torch
    w = synth.WORKLOADS[workload]
    b0 = synth.make_batch(workload, frames=batch)
    code, enc = b0.code, b0.enc
    gcode = D.Code.from_synth(code)
    try:
        from . import autotune
        autotune.apply(gcode, prec, batch)
    except Exception:
        pass
    if precise is not None:   # None: the library's default variable-node form
        gcode.set_tuning(precise=int(precise))
    gcode.set_tuning(quant_bits=quant_bits, quant_step=quant_step)
    dec = D.Decoder(gcode, batch, prec, mode)
    m = code.m
    cw = torch.from_numpy(b0.cw.astype(np.int64)).cuda()
    bits = ((cw[..., None] >> torch.arange(m, device="cuda")) & 1).float()
    x = 1.0 - 2.0 * bits
    gen = torch.Generator(device="cuda")
    out = []
    for pi, e in enumerate(points if points is not None else w["ebn0"]):
        s2 = synth.sigma2_from_ebn0(e, code.design_rate)
        sd = math.sqrt(s2)
        gen.manual_seed(seed * 1000003 + pi)
        frames = errors = bit_errors = 0
        iters_sum = 0
        t0 = time.perf_counter()
        while errors < max_errors and frames < max_frames:
            y = x + sd * torch.randn(x.shape, device="cuda", generator=gen)
            llr = (2.0 / s2) * y
            r = dec(llr.contiguous(), max_iter)
            hard = r["hard"].to(torch.int64)
            wrong = hard != cw
            errors += int(wrong.any(1).sum())
            bit_errors += int(((((hard ^ cw)[..., None] >> torch.arange(m, device="cuda")) & 1)).sum())
            iters_sum += int(r["iters"].sum())
            frames += batch
        lo, hi = wilson(errors, frames)
        res = {"ebn0": e, "prec": prec, "precise": gcode.get_tuning()["precise"], "mode": mode, "quant_bits": quant_bits,
               "quant_step": quant_step / 4096, "frames": frames, "errors": errors, "fer": errors / frames,
               "fer_ci95": [lo, hi], "ber": bit_errors / (frames * code.N * m), "mean_iters": iters_sum / frames,
               "seconds": round(time.perf_counter() - t0, 2)}
        out.append(res)
        if log:
            log(json.dumps(res))
    gcode.close()
    return out


def crossing_db(curve: list[dict], fer: float):
    """Eb/N0 where log10(FER) crosses log10(fer) (linear interpolation between
    the bracketing points); None if the curve does not bracket it."""
    pts = sorted((c["ebn0"], c["fer"]) for c in curve)
    for (e0, f0), (e1, f1) in zip(pts, pts[1:]):
        if f0 >= fer >= f1 and f0 > 0 and f1 > 0 and f0 != f1:
            t = (math.log10(f0) - math.log10(fer)) / (math.log10(f0) - math.log10(f1))
            return e0 + t * (e1 - e0)
    return None


def gap_db(a: list[dict], b: list[dict], fer: float):
    """Eb/N0 of curve b minus that of curve a at frame error rate `fer`."""
    ea, eb = crossing_db(a, fer), crossing_db(b, fer)
    return None if ea is None or eb is None else eb - ea


if __name__ == "__main__":
    import argparse
    ap = argparse.ArgumentParser(description="FER curves of the GPU decoder per storage precision")
    ap.add_argument("--workload", default="gf64_n1000")
    ap.add_argument("--prec", nargs="+", default=["fp32", "fp16"],
                    help="storage precisions; suffix '+p' (fp32+p) selects the FP64 variable node, '+b' the FP32 "
                         "butterfly form; no suffix the library default")
    ap.add_argument("--points", type=float, nargs="*", default=None)
    ap.add_argument("--max-errors", type=int, default=100)
    ap.add_argument("--max-frames", type=int, default=1 << 20)
    ap.add_argument("--target-fer", type=float, default=1e-2)
    ap.add_argument("--mode", default="fused", choices=["fused", "plain", "logsp", "fsp"])
    ap.add_argument("--quant-bits", type=int, default=0, help="emulated b-bit messages (PLAIN, FSP)")
    ap.add_argument("--quant-step", type=int, default=256, help="Log-Fourier magnitude step in units of 2^-12")
    ap.add_argument("--batch", type=int, default=4096)
    a = ap.parse_args()
    curves = {p: fer_curve(a.workload, p.split("+")[0], a.points, a.max_errors, a.max_frames, batch=a.batch,
                           precise={"p": 1, "b": 0}.get(p.split("+")[1]) if "+" in p else None, log=print,
                           mode=a.mode, quant_bits=a.quant_bits,
                           quant_step=a.quant_step) for p in a.prec}
    ref = a.prec[0]
    for p in a.prec[1:]:
        print(json.dumps({"gap_db": gap_db(curves[ref], curves[p], a.target_fer), "ref": ref, "prec": p,
                          "target_fer": a.target_fer}), flush=True)
