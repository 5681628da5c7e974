"""FP64 oracle runs for the long-horizon GPU parity tests: free-running runs
(the oracle's own stop test) that record the fields at checkpoints and the
inner-iteration counts, run on the host's cores (the oracle's per-node
threads for one large lattice, one process per lattice for a batch)."""
import os

import numpy as np

# CPU share of one GPU on the test machines: worker pools and thread counts
# stay within it whatever the host reports
CPU_SHARE = 16


def cpu_share():
    return max(1, min(CPU_SHARE, os.cpu_count() or 1))


def free_run(params, phi0, q0, checkpoints, threads=None):
    """Free-running oracle run; returns ({step: fields}, K history, r history,
    r_prev history)."""
    import oracle
    oracle.set_threads(threads or cpu_share())
    o = oracle.Oracle(params, phi0, q0)
    out = {}
    for T in sorted(checkpoints):
        o.step(T - o.steps_done)
        out[T] = o.fields()
        print(f"  [oracle] {params['nx']}x{params['ny']} step {T}", flush=True)
    res = (out, o.k_history(), o.r_history(), o.r_prev_history())
    o.close()
    return res


def _one(args):
    params, phi0, q0, checkpoints, threads = args
    return free_run(params, phi0, q0, checkpoints, threads)


def free_runs(cases, checkpoints):
    """free_run of every (params, phi0, q0) in cases, one process each, at most
    cpu_share() at a time (largest lattices first).  The workers are fresh
    interpreters (spawned, not forked): they load only numpy and the oracle,
    never the GPU runtime of the calling process."""
    from multiprocessing import get_context
    n = len(cases)
    workers = min(cpu_share(), n)
    threads = max(1, cpu_share() // workers)
    order = sorted(range(n), key=lambda i: -cases[i][0]["nx"] * cases[i][0]["ny"])
    with get_context("spawn").Pool(workers) as pool:
        res = pool.map(_one, [(*cases[i], checkpoints, threads) for i in order], chunksize=1)
    out = [None] * n
    for k, i in enumerate(order):
        out[i] = res[k]
    return out


def replay_counts(K, steps):
    """presolve_iters and the per-step counts of the first `steps` steps of an
    oracle K history (entry 0 is the initial solve)."""
    return int(K[0]), np.ascontiguousarray(K[1:steps + 1], dtype=np.int32)
