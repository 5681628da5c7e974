"""Throughput of the coupled two-phase EHD lattice Boltzmann step on one MI355X.

Workload: the batched droplet sweep (512 independent drops, square lattices of
side 64..384, seeded), all instances advanced together in device-steered
rounds over one tile work list (hipGraph-captured chunks) with FP16-shifted
population storage.  One "step" is one outer step of Algorithm 1 for every
instance (main pass + inner potential loop).  Beside it the same workload with
FP32 storage, a subset run instance by instance through the FP32
single-instance path, and the FP64 oracle timed on the host.

The roofline object is for the dominant kernel, the round kernel: algorithmic
bytes of a timed stretch of steps divided by the summed duration of its round
launches, each bracketed by HIP events on the library's stream.

Prints one JSON line (rank 0, N = 1).
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
# algorithmic bytes per lattice update (read + write of populations and
# auxiliary fields): main pass, and one inner potential iteration
ALGO_BYTES = {"fp32": (276.0, 88.0), "fp16s": (180.0, 56.0)}
METRIC = "coupled-step MLUPS + HBM GB/s (% peak), batched FP16-store vs FP32 plain"


def src_digest():
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2407_01654_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources."""
    for f in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(f):
            if line.startswith("bench-traffic:"):
                try:
                    d = json.loads(line.split(":", 1)[1])
                except json.JSONDecodeError:
                    continue
                if d.get("kernel") == kernel and d.get("src_sha") == src_digest():
                    return d
    return None


def build_workload(n_inst, seed):
    from paper_2407_01654_amd import workloads as W
    return W.batch_sweep(n_inst=n_inst, seed=seed)


def make_sim(wls, prec, launch):
    from paper_2407_01654_amd import lbm
    return lbm.Simulation([w.params for w in wls], [w.phi0 for w in wls], [w.q0 for w in wls],
                          prec=prec, launch=launch)




def timed_run(sim, wls, steps, warmup, calls):
    """Times `steps` outer steps in `calls` step() calls after `warmup` steps.
    Returns the wall time, per-call event times and the lattice work done."""
    import torch
    n = len(wls)
    nodes = np.array([w.params["nx"] * w.params["ny"] for w in wls], dtype=np.float64)
    if warmup:
        sim.step(warmup)
    sim.sync()
    k0 = [sim.stats(i)["total_iters"] for i in range(n)]
    stream = torch.cuda.current_stream()
    per = [steps // calls + (1 if c < steps % calls else 0) for c in range(calls)]
    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in per:
        if k == 0:
            continue
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        sim.step(k)
        b.record(stream)
        ev.append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    st = sim.sync()
    k1 = [sim.stats(i)["total_iters"] for i in range(n)]
    # inner iterations in the timed region, weighted by lattice size
    kn = float(sum((k1[i] - k0[i]) * nodes[i] for i in range(n)))
    return dict(wall=wall, call_ms=[a.elapsed_time(b) for a, b in ev], nodes=float(nodes.sum()),
                iter_nodes=kn, mean_k=kn / (nodes.sum() * steps), status=st)


def kernel_timing(sim, wls, steps):
    """Per-launch durations of the round and finalize kernels over `steps`
    further steps, and the algorithmic work of those steps."""
    n = len(wls)
    nodes = np.array([w.params["nx"] * w.params["ny"] for w in wls], dtype=np.float64)
    sim.sync()
    k0 = [sim.stats(i)["total_iters"] for i in range(n)]
    sim.timing(True)
    sim.step(steps)
    t = sim.timing(False)
    k1 = [sim.stats(i)["total_iters"] for i in range(n)]
    t["iter_nodes"] = float(sum((k1[i] - k0[i]) * nodes[i] for i in range(n)))
    t["main_nodes"] = float(nodes.sum()) * steps
    return t


def cpu_baseline(wls, budget_s=15.0):
    """FP64 oracle on the host: instances of the same sweep, one after the
    other, each for a few steps with its inner loop replayed at one iteration
    per step (the steady regime), until about budget_s of CPU time."""
    import oracle
    oracle.build(force=False)
    done_nodes = 0.0
    t0 = time.process_time()
    used = []
    for w in wls:
        p = dict(w.params, presolve_iters=1)
        o = oracle.Oracle(p, w.phi0, w.q0)
        o.set_replay(np.ones(4, dtype=np.int32))
        o.step(4)
        done_nodes += 4.0 * p["nx"] * p["ny"]
        used.append(p["nx"])
        if time.process_time() - t0 > budget_s:
            break
    dt = time.process_time() - t0
    return {"value": done_nodes / dt / 1e6, "unit": "MLUPS", "cores": 1, "kind": "oracle",
            "sample": f"{len(used)} instances of the sweep (sides {sorted(set(used))}), 4 steps each, "
                      f"inner loop replayed at 1 iteration/step; {dt:.1f} s single-threaded"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--instances", type=int, default=512)
    ap.add_argument("--calls", type=int, default=4, help="step() calls the timed steps are split into")
    ap.add_argument("--band-y", type=int, default=64)
    ap.add_argument("--timing-steps", type=int, default=10)
    ap.add_argument("--single-subset", type=int, default=16)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", choices=["fp16s", "fp32", "all"], default="all")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU: the batched sweep would shard by instance "
                                   "across GPUs, which is not implemented; run with --gpus 1"}))
        sys.exit(2)
    import torch
    from paper_2407_01654_amd import lbm
    lbm.load()
    torch.cuda.set_device(0)

    wls = build_workload(args.instances, seed=4)
    launch = dict(block_x=64, band_y=args.band_y, device_loop=1, rounds_per_graph=0)
    res, ktime = {}, {}
    for prec in (("fp16s", "fp32") if args.only == "all" else (args.only,)):
        print(f"[bench] batched {prec}: init", file=sys.stderr, flush=True)
        sim = make_sim(wls, prec, launch)
        print(f"[bench] batched {prec}: warmup {args.warmup}, timed {args.steps}", file=sys.stderr, flush=True)
        res[prec] = timed_run(sim, wls, args.steps, args.warmup, args.calls)
        print(f"[bench] batched {prec}: kernel timing over {args.timing_steps} steps", file=sys.stderr, flush=True)
        ktime[prec] = kernel_timing(sim, wls, args.timing_steps)
        del sim
        torch.cuda.empty_cache()

    single = None
    if args.only == "all" and args.single_subset > 0:
        print(f"[bench] fp32 single-instance path on {args.single_subset} instances", file=sys.stderr, flush=True)
        tot_t, tot_n = 0.0, 0.0
        for w in wls[:args.single_subset]:
            sim = make_sim([w], "fp32", launch)
            r = timed_run(sim, [w], args.steps, args.warmup, args.calls)
            tot_t += r["wall"]
            tot_n += r["nodes"] * args.steps
            del sim
        single = tot_n / tot_t / 1e6

    head_prec = "fp16s" if "fp16s" in res else "fp32"
    head, kt = res[head_prec], ktime[head_prec]
    steps = args.steps
    mlups = head["nodes"] * steps / head["wall"] / 1e6
    main_b, pot_b = ALGO_BYTES[head_prec]
    algo_bytes = kt["main_nodes"] * main_b + kt["iter_nodes"] * pot_b
    n_launch = kt["round_launches"]
    avg_launch_s = kt["round_ms"] * 1e-3 / n_launch
    achieved = algo_bytes / n_launch / avg_launch_s / 1e9
    kname = f"k_round<{'StoreF16S' if head_prec == 'fp16s' else 'StoreF32'}>"
    tr = stored_traffic(kname)
    traffic = None
    if tr is not None and tr.get("band_y") == args.band_y and tr.get("instances") == args.instances:
        traffic = tr["bytes_per_launch"]
    out = {
        "metric": METRIC,
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["wall"] / steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"batched droplet sweep: {args.instances} drops, sides 64-384 (seed 4), "
                        f"{head_prec} population storage, device-steered rounds in hipGraph chunks",
            "instances": args.instances, "lattice_nodes": int(head["nodes"]),
            "storage": head_prec, "block_x": launch["block_x"], "band_y": launch["band_y"],
            "step_calls": args.calls, "mean_inner_iters": round(head["mean_k"], 3),
        },
        "hbm_gbs_algorithmic": round(algo_bytes / (kt["round_ms"] + kt["finalize_ms"]) / 1e6, 1),
        "roofline": {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
            "kernel": kname,
            "algorithmic_bytes_per_lup": {"main": main_b, "per_inner_iteration": pot_b},
            "avg_launch_ms": round(avg_launch_s * 1e3, 4), "launches_timed": n_launch,
            "finalize_avg_ms": round(kt["finalize_ms"] / max(kt["finalize_launches"], 1), 4),
        },
    }
    if "fp32" in res and "fp16s" in res:
        r32 = res["fp32"]
        out["fp32_batched_mlups"] = round(r32["nodes"] * steps / r32["wall"] / 1e6, 1)
        out["fp16s_over_fp32_batched"] = round(mlups / out["fp32_batched_mlups"], 3)
        k32 = ktime["fp32"]
        b32 = k32["main_nodes"] * ALGO_BYTES["fp32"][0] + k32["iter_nodes"] * ALGO_BYTES["fp32"][1]
        out["fp32_round_kernel_gbs"] = round(b32 / k32["round_ms"] / 1e6, 1)
    if single is not None:
        out["fp32_single_instance_mlups"] = round(single, 1)
        out["batched_fp16s_over_fp32_single"] = round(mlups / single, 3)
        out["single_subset"] = args.single_subset
    if not args.no_cpu:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(wls)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
