"""Oracle traces of selected pairs, computed in parallel CPU processes.

Each worker draws its pair with the oracle's own sampler (from the seed and
the global pair index, never from the device) and contracts it with the
dense or the MPO-zip oracle.  Spawned processes do not touch the GPU.
"""

import multiprocessing as mp
import os


def _one(job):
    ansatz, n, depth, seed, pair, fp32, method = job
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except Exception:
        pass
    from oracle import dense, mpo, sampler
    pr = sampler.sample_pairs(ansatz, n, depth, seed, pair, 1, fp32=fp32)
    mod = dense if method == "dense" else mpo
    return complex(mod.traces(pr)[0])


def workers():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def traces(ansatz, n, depth, seed, pairs, fp32, method="mpo"):
    """Oracle Tr(U^dagger V) of global pairs `pairs` (a list of indices)."""
    jobs = [(ansatz, n, depth, seed, int(p), bool(fp32), method) for p in pairs]
    if len(jobs) <= 1:
        return [_one(j) for j in jobs]
    with mp.get_context("spawn").Pool(min(workers(), len(jobs))) as pool:
        return pool.map(_one, jobs, chunksize=1)
