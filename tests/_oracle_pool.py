"""The FP64 oracle's decode of a frame sample spread over host processes (the
oracle is single-threaded NumPy; frames are independent).  Spawned workers
never touch the GPU."""
import multiprocessing as mp
import os

import numpy as np


def _worker(args):
    arrays, llr, max_iter = args
    from oracle.sp import TannerCode, decode
    tc = TannerCode(*arrays)
    r = decode(tc, llr, max_iter)
    return r.hard, r.iters, r.converged


def oracle_decode_sample(code, llr, max_iter, workers=None):
    """Oracle hard decisions, iteration counts and convergence flags of llr
    [n, N, m] (n frames of `code`, a synth code), n split over the workers."""
    n = llr.shape[0]
    workers = max(1, min(workers or min(16, os.cpu_count() or 1), n))
    arrays = (code.M, code.N, code.m, code.row_ptr, code.col, code.val, code.poly)
    parts = np.array_split(np.arange(n), workers)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS"):
        os.environ.setdefault(k, "1")
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_worker, [(arrays, llr[p], max_iter) for p in parts])
    hard = np.concatenate([r[0] for r in res])
    iters = np.concatenate([r[1] for r in res])
    conv = np.concatenate([r[2] for r in res])
    return hard, iters, conv
