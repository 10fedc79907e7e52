"""Benchmark of the MI355X Swendsen-Wang engine.

Default workload: 2D q=3 Potts and 2D Ising, L = 4096, periodic, at their
exact critical temperatures, hot start, plain form (one lattice per launch).
A step is one SW sweep of every lattice of the workload (bond generation +
tile labelling, label merge, cluster flip, per-sweep measurement).  Prints one
JSON line with spin updates/ns, the HBM roofline of the dominant kernel and
the oracle timed on the host as a CPU baseline.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C2|C1|C3|C4|C5]

C5 is the served form: a seeded Poisson job mix (--jobs, --rate) replayed in
wall-clock time against the continuous-batching server, reporting served
throughput, p50/p99 job latency (arrival to last sweep) and the same jobs
run back to back in the plain form.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, 8 TB/s
KERNELS = ("bond", "merge", "flip")

WORKLOADS = {
    "C1": ["C1"],
    "C2": ["C2-potts", "C2-ising"],
    "C2-8192": ["C2-potts-8192", "C2-ising-8192"],
    "C3": ["C3"],
    "C4": ["C4"],
    "C5": [],
}
DESCRIPTION = {
    "C1": "2D Ising L=64 T=2.269185 seed 1, plain form",
    "C2": "2D q=3 Potts + 2D Ising, L=4096, exact Tc, plain form (one lattice per launch)",
    "C2-8192": "2D q=3 Potts + 2D Ising, L=8192, exact Tc, plain form (working set above the 256 MB Infinity Cache)",
    "C3": "3D Ising L=256 T=4.5115, plain form",
    "C4": "3D XY L=128, 32 replicas over [0.95 Tc, 1.05 Tc], batched form",
    "C5": "served job mix (2D Ising, 2D Potts q in {3,4,10}, 3D Ising, 3D XY; L log-uniform; "
          "100-5000 sweeps), Poisson arrivals, continuous batching",
}


def algorithmic_bytes_per_site(model):
    # k_bond applies the previous sweep's cluster decisions as it reads the
    # incoming configuration: it reads the previous sweep's int32 label and
    # writes the bond byte and the new int32 label; XY also reads the
    # previous working angle and writes the new one (FP32).
    return 4 + 1 + 4 + (8 if model == 2 else 0)


def kernel_source_hash():
    src = os.path.join(ROOT, "paper_1403_7560_amd", "csrc", "sw_kernels.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(config, bytes_per_launch_alg):
    """HBM bytes per k_bond launch from the committed rocprofv3 counter runs,
    or None when they were taken on another version of the kernels."""
    path = os.path.join(ROOT, "profiles", f"k_bond_traffic_{config}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_hash") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(config, lattices):
    """The oracle (single-threaded C) on a bounded sample of the workload."""
    import numpy as np
    import oracle
    if config == "C4":
        lattices = lattices[:1]
    sweeps = 200 if config == "C1" else 1
    t0 = time.perf_counter()
    updates = 0
    for j in lattices:
        s0 = oracle.init_state(j["model"], j["dim"], j["L"], j["q"], j["seed"], j["replica"])
        oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], 0,
                      sweeps, s0, record=True, last=False)
        updates += j["L"] ** j["dim"] * sweeps
    dt = time.perf_counter() - t0
    names = ", ".join(f"{'Ising' if j['model'] == 0 else 'Potts' if j['model'] == 1 else 'XY'}"
                      f" {j['dim']}D L={j['L']}" for j in lattices)
    return {"value": updates / (dt * 1e9), "unit": "spin updates/ns", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} sweep(s) from hot start of each of: {names}; {dt:.1f} s"}


def served(n_jobs, rate, seed=2014, plain=True):
    """Replay the job mix against the server; then (unless plain is False)
    the same jobs in the plain form, one after another."""
    import numpy as np
    import paper_1403_7560_amd as sw
    from paper_1403_7560_amd import inputs
    jobs = inputs.job_mix(n_jobs, rate=rate, seed=seed)
    updates = sum(j["L"] ** j["dim"] * j["sweeps"] for j in jobs)
    srv = sw.Server(96 << 30, max_active=256, chunk=32)
    lat_s = np.zeros(n_jobs)
    finish = np.zeros(n_jobs)
    info = {}
    pending = set()
    i = 0
    t0 = time.perf_counter()
    while len(info) < n_jobs or pending:
        now = time.perf_counter() - t0
        while i < n_jobs and jobs[i]["arrival"] <= now:
            j = jobs[i]
            jid = srv.submit(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], 0, j["sweeps"])
            info[jid] = (i, time.perf_counter() - t0 - j["arrival"])
            pending.add(jid)
            i += 1
        left = srv.step()
        for jid in list(pending):
            r = srv.poll(jid)
            if r is None:
                continue
            if r["status"] != 0:
                raise RuntimeError(f"job {jid} failed with status {r['status']}")
            k, delay = info[jid]
            lat_s[k] = (r["finish_s"] - r["submit_s"]) + delay
            finish[k] = time.perf_counter() - t0
            pending.discard(jid)
        if left == 0 and i < n_jobs:
            time.sleep(max(0.0, jobs[i]["arrival"] - (time.perf_counter() - t0)))
    makespan = finish.max() - jobs[0]["arrival"]
    srv.close()
    value = updates / (makespan * 1e9)
    offered = updates / ((jobs[-1]["arrival"] - jobs[0]["arrival"]) * 1e9)
    out = {
        "value": value, "makespan_s": makespan, "updates": updates,
        "latency_s": {"p50": round(float(np.percentile(lat_s, 50)), 4),
                      "p99": round(float(np.percentile(lat_s, 99)), 4),
                      "max": round(float(lat_s.max()), 4)},
        "offered_load": round(offered, 2),
        # above 1 the queue grows over the trace: latencies then depend on its length
        "offered_over_served": round(offered / value, 3),
        "plain_form": None, "speedup_vs_plain": None,
    }
    if plain:
        t1 = time.perf_counter()
        for j in jobs:
            lat = sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"])
            lat.sweep(j["sweeps"])
            lat.close()
        plain_s = time.perf_counter() - t1
        pv = updates / (plain_s * 1e9)
        out["plain_form"] = {"value": round(pv, 3), "seconds": round(plain_s, 2)}
        out["speedup_vs_plain"] = round(value / pv, 3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="C2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--jobs", type=int, default=300, help="C5: jobs in the replayed trace")
    ap.add_argument("--rate", type=float, default=200.0, help="C5: arrivals per second")
    ap.add_argument("--no-plain", action="store_true", help="C5: skip the plain-form replay of the same jobs")
    ap.add_argument("--copy-probe", type=int, default=0,
                    help="also copy this many bytes device-to-device once (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this engine runs on one GPU only; --gpus {args.gpus} is not supported "
              "(independent lattices shard across GPUs, one process per GPU)",
              file=sys.stderr)
        sys.exit(2)

    import paper_1403_7560_amd as sw
    from paper_1403_7560_amd import inputs

    if args.copy_probe:
        # a plain copy of known size: reads and writes copy_probe bytes, for
        # scaling the HBM byte counters of the profiler
        import torch
        a = torch.ones(args.copy_probe // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.config == "C5":
        r = served(args.jobs, args.rate, plain=not args.no_plain)
        out = {
            "metric": "spin updates/ns", "value": round(r["value"], 3), "unit": "spin updates/ns",
            "n_gpus": 1, "steps": args.jobs, "warmup": 0,
            "ms_per_step": round(r["makespan_s"] * 1e3 / args.jobs, 4),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
            "data": "synthetic",
            "config": {"workload": f"C5: {DESCRIPTION['C5']}", "jobs": args.jobs, "rate_per_s": args.rate,
                       "updates": r["updates"], "offered_load_updates_per_ns": r["offered_load"],
                       "offered_over_served": r["offered_over_served"],
                       "step": "one served job"},
            "latency_s": r["latency_s"], "plain_form": r["plain_form"],
            "speedup_vs_plain": r["speedup_vs_plain"],
            "roofline": None, "cpu_baseline": None,
        }
        print(json.dumps(out), flush=True)
        return

    lattices = []
    default_steps = None
    for name in WORKLOADS[args.config]:
        lats, n = inputs.workload(name)
        lattices += lats
        default_steps = n
    K = args.steps if args.steps is not None else default_steps
    W = args.warmup

    prof = {k: [0.0, 0] for k in KERNELS}
    alg_bytes = 0
    n_bond = 0
    if args.config == "C4":
        b = sw.Batch(lattices)
        b.sweep(W)
        t0 = time.perf_counter()
        b.sweep(K)
        dt = time.perf_counter() - t0
        total = sum(j["L"] ** j["dim"] for j in lattices) * K
        roof = None
    else:
        lats = [sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"])
                for j in lattices]
        for lat in lats:
            lat.sweep(W)
        for lat in lats:
            lat.profile(1)  # HIP events around the k_bond launch of every 16th sweep of the timed region
        t0 = time.perf_counter()
        for lat in lats:
            lat.sweep(K)
        dt = time.perf_counter() - t0
        total = 0
        for lat in lats:
            p = lat.profile_read()
            lat.profile(0)
            for k in KERNELS:
                prof[k][0] += p[k][0]
                prof[k][1] += p[k][1]
            total += lat.N * K
            # the timed launches only (every 16th sweep)
            alg_bytes += algorithmic_bytes_per_site(lat.model) * lat.N * p["bond"][1]
            n_bond += p["bond"][1]
        bond_ms = prof["bond"][0]
        achieved = alg_bytes / (bond_ms * 1e-3) / 1e9
        per_launch = alg_bytes / max(n_bond, 1)
        roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(args.config, per_launch),
                "kernel": "k_bond (bond generation + tile labelling)",
                "algorithmic_bytes_per_launch": per_launch,
                "avg_launch_us": round(bond_ms * 1e3 / max(n_bond, 1), 2),
                "kernel_avg_us": {k: round(prof[k][0] * 1e3 / prof[k][1], 2) for k in KERNELS if prof[k][1]}}

    value = total / (dt * 1e9)
    models = sorted({j["model"] for j in lattices})
    out = {
        "metric": "spin updates/ns",
        "value": round(value, 3),
        "unit": "spin updates/ns",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(dt * 1e3 / K, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if models == [2] else "u32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {DESCRIPTION[args.config]}",
                   "lattices": [{k: j[k] for k in ("model", "dim", "L", "q", "beta", "seed", "replica")}
                                for j in lattices[:4]] + ([f"... {len(lattices)} lattices"]
                                                          if len(lattices) > 4 else []),
                   "sweeps_per_lattice": K},
        "roofline": roof,
        "cpu_baseline": None if args.no_cpu_baseline else cpu_baseline(args.config, lattices),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
