"""Writes config5_horizon.npz: the FP64 oracle's free-running run of the
2048 x 4096 sessile drop (config 5), sampled every `every` steps up to
`steps` for the long-horizon parity test of the GPU path.

Everything stored comes from the oracle (its own stop test of Algorithm 1
step 3, run on this host's cores): the per-step inner-iteration counts (the
GPU replays them), and at each checkpoint the fields phi, psi, rho_e, ux, uy
and p on three lines through the drop (the column x = 1024 through its
centre, the row y = 128 through it, the row y = 320 above it) and on 4096
seeded random nodes, with each field's mean and maximum magnitude over the
whole lattice (for p, of p minus its mean), which the test normalises by.
The sampled values are stored rounded to float32 (relative rounding 6e-8,
far below the 1e-5 bar); the scalars and counts exactly.  The file is
rewritten at every checkpoint.

Run from the repository root:
  python3 tests/golden/make_config5_horizon.py [steps [every]]
(defaults 10000 and 1000; about 0.9 s per step on 8 cores).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2407_01654_amd import workloads as W  # noqa: E402

FIELDS = ("phi", "psi", "rho_e", "ux", "uy", "p")
COLUMN_X, ROWS_Y = 1024, (128, 320)
N_RANDOM, SEED = 4096, 5


def sample_index(nx, ny):
    rng = np.random.default_rng(SEED)
    ry = rng.integers(0, ny, N_RANDOM)
    rx = rng.integers(0, nx, N_RANDOM)
    return ry, rx


def main(steps=10000, every=1000, out=os.path.join(ROOT, "tests", "golden", "config5_horizon.npz")):
    checkpoints = tuple(range(every, steps + 1, every))
    wl = W.sessile_drop()
    nx, ny = wl.params["nx"], wl.params["ny"]
    ry, rx = sample_index(nx, ny)
    t0 = time.time()
    ora = oracle.Oracle(wl.params, wl.phi0, wl.q0)
    print(f"[c5] oracle ready in {time.time() - t0:.0f} s, {oracle.max_threads()} threads", flush=True)
    data = {"random_y": ry, "random_x": rx, "column_x": np.array(COLUMN_X), "rows_y": np.array(ROWS_Y)}
    done = 0
    for T in checkpoints:
        ora.step(T - done)
        done = T
        f = ora.fields()
        for k in FIELDS:
            a = f[k]
            data[f"{T}/{k}/column"] = a[:, COLUMN_X].astype(np.float32)
            for y in ROWS_Y:
                data[f"{T}/{k}/row{y}"] = a[y, :].astype(np.float32)
            data[f"{T}/{k}/random"] = a[ry, rx].astype(np.float32)
            m = a.mean()
            # p is compared after removing its mean, so its scale is that of p - mean
            data[f"{T}/{k}/absmax"] = np.array(np.abs(a - m).max() if k == "p" else np.abs(a).max())
            data[f"{T}/{k}/mean"] = np.array(m)
        data["checkpoints"] = np.array([t for t in checkpoints if t <= T])
        data["k_history"] = ora.k_history().astype(np.int32)
        tmp = out + ".tmp.npz"
        np.savez_compressed(tmp, **data)
        os.replace(tmp, out)
        print(f"[c5] step {T} after {time.time() - t0:.0f} s, wrote {out}", flush=True)


if __name__ == "__main__":
    main(*(int(a) for a in sys.argv[1:3]))
