"""Benchmark of the MI355X Swendsen-Wang engine.

Default workload: 2D q=3 Potts and 2D Ising, L = 4096, periodic, at their
exact critical temperatures, hot start, plain form (one lattice per launch).
A step is one SW sweep of every lattice of the workload (bond generation +
tile labelling, label merge, cluster flip, per-sweep measurement).  Prints one
JSON line with spin updates/ns, the HBM roofline of the dominant kernel, a
per-kernel block (bond, global labelling, flip), the oracle timed on the
host's cores as a CPU baseline, and compact figures of the other workloads:
3D Ising L=256 (plain), 3D XY 32 x 128^3 (batched), the paper's 512-state
clock model on its Table 2 shape (3D L=256), and the served job mix (at the
configured 200 jobs/s and at a rate the server sustains, with the same jobs
run back to back in the plain form).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config C2|C1|C3|C4|C5|CLOCK]
                    [--labeller 0|1|2] [--quick]

C5 alone is the served form: a seeded Poisson job mix (--jobs, --rate)
replayed in wall-clock time against the continuous-batching server,
reporting served throughput, p50/p99 job latency (arrival to last sweep) and
the same jobs run back to back in the plain form.
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
    "CLOCK": ["CLOCK-512"],
}
DESCRIPTION = {
    "C1": "2D Ising L=64 T=2.269185 seed 1, plain form",
    "C2": "2D q=3 Potts + 2D Ising, L=4096, exact Tc, plain form (one lattice per launch)",
    "C2-8192": "2D q=3 Potts + 2D Ising, L=8192, exact Tc, plain form (working set above the 256 MB Infinity Cache)",
    "C3": "3D Ising L=256 T=4.5115, plain form",
    "C4": "3D XY L=128, 32 replicas over [0.95 Tc, 1.05 Tc], batched form",
    "C5": "served job mix (2D Ising, 2D Potts q in {3,4,10}, 3D Ising, 3D XY; L log-uniform; "
          "100-5000 sweeps), Poisson arrivals, continuous batching",
    "CLOCK": "3D 512-state clock model L=256 T=2.20175 (the paper's Table 2 shape), plain form",
}
# the paper's own figures for the same shapes (GTX580, update + measurement
# rows of Tables 1 and 2): context only, another machine
PAPER_CONTEXT = {
    "C3": {"updates_per_ns": 0.300, "source": "Table 1, 3D Ising L=256, update + measurement, GTX580"},
    "CLOCK": {"updates_per_ns": 0.223, "source": "Table 2, 3D XY (q=512 clock) L=256, update + measurement, GTX580"},
}


def algorithmic_bytes_per_site(model):
    # k_bond applies the previous sweep's cluster decisions as it reads the
    # incoming configuration: it reads the previous sweep's int32 label and
    # writes the bond byte and the new int32 label; XY also reads the
    # previous working angle and writes the new one (FP32), the clock model
    # its state index (16 bits).
    return 4 + 1 + 4 + {2: 8, 3: 4}.get(model, 0)


def flip_bytes_per_site(model):
    # k_flip reads the label word and writes the state (1 B; the clock model
    # reads its working state index and writes the state, 2 + 2 B; XY 4 + 4 B)
    return 4 + {2: 8, 3: 4}.get(model, 1)


def merge_bytes_per_launch(lat):
    # the global phase reads both sides of every tile face (two int32 slots
    # per face element); the label words it touches are a few per cluster
    # crossing a face, not counted
    return 8 * lat.face_elements()


def copy_probe(sw, nbytes):
    """One device-to-device copy of nbytes (the runtime's copy kernel reads
    and writes nbytes), for scaling the profiler's HBM byte counters.  It
    goes through the HIP runtime the engine's library itself loaded (found
    by its soname once the library is in), so that the probe and the
    kernels it calibrates run on the same runtime."""
    import ctypes
    sw.lib()
    hip = ctypes.CDLL("libamdhip64.so.7")
    a, b = ctypes.c_void_p(), ctypes.c_void_p()
    n = ctypes.c_size_t(nbytes)
    for rc in (hip.hipMalloc(ctypes.byref(a), n), hip.hipMalloc(ctypes.byref(b), n),
               hip.hipMemset(a, 1, n), hip.hipDeviceSynchronize(),
               hip.hipMemcpy(b, a, n, 3),  # hipMemcpyDeviceToDevice
               hip.hipDeviceSynchronize(), hip.hipFree(a), hip.hipFree(b)):
        if rc != 0:
            raise RuntimeError(f"copy probe: HIP error {rc}")


def job_hbm(bond_bytes, seconds):
    """Whole-job HBM figure of a form (plain, batched, served): the bond
    kernel's algorithmic bytes of every sweep run (the dominant kernel; the
    global phase and the flip add a few percent) over the wall time."""
    gbs = bond_bytes / seconds / 1e9
    return {"achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "bytes": "bond-kernel algorithmic bytes of every sweep / wall time"}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("sw_bond.h", "sw_device.h", "sw_internal.h"):
        with open(os.path.join(ROOT, "paper_1403_7560_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


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


def _oracle_sample(args):
    """One oracle chain (a worker of the CPU baseline): sweeps from the hot
    start of lattice j; returns (updates, seconds)."""
    j, sweeps = args
    import oracle
    s0 = oracle.init_state(j["model"], j["dim"], j["L"], j["q"], j["seed"], j["replica"])
    t0 = time.perf_counter()
    oracle.sweeps(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"], 0,
                  sweeps, s0, record=True, last=False)
    return j["L"] ** j["dim"] * sweeps, time.perf_counter() - t0


def cpu_baseline(config, lattices):
    """The oracle (single-threaded C, as it stands) on a bounded sample of the
    workload: first one chain on one core, then one independent chain per
    host core at once (replicas with their own replica index), whose
    aggregate rate is the baseline.  Runs before anything touches the GPU:
    the workers are forked."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    if config == "C4":
        lattices = lattices[:1]
    sweeps = 200 if config == "C1" else 1
    names = ", ".join(f"{['Ising', 'Potts', 'XY', 'clock'][j['model']]} {j['dim']}D L={j['L']}" for j in lattices)
    one = [_oracle_sample((j, sweeps)) for j in lattices]
    v1 = sum(u for u, _ in one) / (sum(t for _, t in one) * 1e9)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    jobs = [(dict(lattices[r % len(lattices)], replica=1000 + r), sweeps) for r in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_oracle_sample, jobs)
    wall = time.perf_counter() - t0
    upd = sum(u for u, _ in res)
    return {"value": upd / (wall * 1e9), "unit": "spin updates/ns", "cores": cores, "kind": "oracle",
            "sample": f"{cores} independent oracle chains at once, one per host core, each {sweeps} sweep(s) "
                      f"from the hot start of one of: {names}; {wall:.1f} s wall",
            "one_core": {"value": v1, "cores": 1, "seconds": round(sum(t for _, t in one), 2)}}


def served(n_jobs, rate, seed=2014, plain=True):
    """Replay the job mix against the server; then (unless plain is False)
    the same jobs in the plain form, one after another."""
    import numpy as np
    import paper_1403_7560_amd as sw
    from paper_1403_7560_amd import inputs
    jobs = inputs.job_mix(n_jobs, rate=rate, seed=seed)
    updates = sum(j["L"] ** j["dim"] * j["sweeps"] for j in jobs)
    bond_bytes = sum(j["L"] ** j["dim"] * j["sweeps"] * algorithmic_bytes_per_site(j["model"]) for j in jobs)
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
        "job_hbm": job_hbm(bond_bytes, makespan),
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
        out["plain_form"] = {"value": round(pv, 3), "seconds": round(plain_s, 2),
                             "job_hbm": job_hbm(bond_bytes, plain_s)}
        out["speedup_vs_plain"] = round(value / pv, 3)
    return out


def timed_plain(sw, lattices, W, K, labeller=None, measure=True):
    """W warm-up and K timed sweeps of each lattice in the plain form, with
    HIP events (profile level 2) around the bond kernel and the global
    labelling phase of every 16th sweep and around each call's flip.
    measure=False switches the per-sweep observables off (the paper's
    "update" rows against "update + measurement").
    Returns (updates/ns, seconds, per-kernel block, lattices)."""
    lats = [sw.Lattice(j["model"], j["dim"], j["L"], j["q"], j["beta"], j["seed"], j["replica"])
            for j in lattices]
    if not measure:
        for lat in lats:
            lat.set_measure(False)
    if labeller is not None:
        for lat in lats:
            lat.set_labeller(labeller, 256)
    for lat in lats:
        lat.sweep(W)
    for lat in lats:
        lat.profile(2)
    t0 = time.perf_counter()
    for lat in lats:
        lat.sweep(K)
    dt = time.perf_counter() - t0
    total = 0
    kb = {"k_bond": [0.0, 0, 0.0], "global_phase": [0.0, 0, 0.0], "k_flip": [0.0, 0, 0.0]}  # ms, launches, bytes
    for lat in lats:
        p = lat.profile_read()
        lat.profile(0)
        total += lat.N * K
        for name, key, per in (("k_bond", "bond", algorithmic_bytes_per_site(lat.model) * lat.N),
                               ("global_phase", "merge", merge_bytes_per_launch(lat)),
                               ("k_flip", "flip", flip_bytes_per_site(lat.model) * lat.N)):
            kb[name][0] += float(p[key][0])
            kb[name][1] += int(p[key][1])
            kb[name][2] += float(per) * int(p[key][1])
    if labeller in (0, 1):
        st = [lat.label_stats() for lat in lats]
        n_lab = sum(x["labellings"] for x in st)
        kb_scans = {"scans_per_sweep": round(sum(x["scans"] for x in st) / max(n_lab, 1), 2),
                    "max_scans": max(x["max_scans"] for x in st)}
    else:
        kb_scans = None
    kernels = {}
    for name, (ms, n, byts) in kb.items():
        if n == 0:
            continue
        gbs = byts / (ms * 1e-3) / 1e9
        kernels[name] = {"avg_us": round(ms * 1e3 / n, 2), "launches_timed": int(n),
                         "algorithmic_bytes_per_launch": int(byts / n),
                         "achieved_GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    if kb_scans and "global_phase" in kernels:
        kernels["global_phase"].update(kb_scans)
    return total / (dt * 1e9), dt, kernels, lats


def leg_plain(sw, inputs, name, W, K, labeller=None):
    lattices, _ = inputs.workload(name)
    v, dt, kernels, lats = timed_plain(sw, lattices, W, K, labeller)
    for lat in lats:
        lat.close()
    bond_bytes = sum(j["L"] ** j["dim"] * algorithmic_bytes_per_site(j["model"]) for j in lattices) * K
    return {"value": round(v, 3), "unit": "spin updates/ns", "ms_per_sweep": round(dt * 1e3 / K, 4),
            "steps": K, "warmup": W, "kernels": kernels, "job_hbm": job_hbm(bond_bytes, dt)}


def update_only(sw, lattices, W, K):
    """The plain-form leg of these lattices with the per-sweep measurement
    switched off."""
    v, dt, kernels, lats = timed_plain(sw, lattices, W, K, measure=False)
    for lat in lats:
        lat.close()
    return {"value": round(v, 3), "ms_per_sweep": round(dt * 1e3 / K, 4),
            "k_bond_us": (kernels or {}).get("k_bond", {}).get("avg_us")}


def leg_batched(sw, inputs, name, W, K):
    lattices, _ = inputs.workload(name)
    b = sw.Batch(lattices)
    b.sweep(W)
    t0 = time.perf_counter()
    b.sweep(K)
    dt = time.perf_counter() - t0
    b.close()
    total = sum(j["L"] ** j["dim"] for j in lattices) * K
    bond_bytes = sum(j["L"] ** j["dim"] * algorithmic_bytes_per_site(j["model"]) for j in lattices) * K
    return {"value": round(total / (dt * 1e9), 3), "unit": "spin updates/ns",
            "ms_per_step": round(dt * 1e3 / K, 4), "steps": K, "warmup": W, "lattices": len(lattices),
            "job_hbm": job_hbm(bond_bytes, dt)}


def to_json(out):
    # numpy scalars (from the binding's arrays) as plain numbers
    return json.dumps(out, default=lambda o: o.item() if hasattr(o, "item") else str(o))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--config", default="C2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--quick", action="store_true", help="skip the secondary workloads of the default line")
    ap.add_argument("--labeller", type=int, default=None, choices=(0, 1, 2),
                    help="plain form: global labelling phase (0 Hawick, 1 Kalentev, 2 union)")
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

    from paper_1403_7560_amd import inputs
    lattices = []
    default_steps = None
    for name in WORKLOADS[args.config]:
        lats, n = inputs.workload(name)
        lattices += lats
        default_steps = n
    # the CPU baseline forks its workers, so it runs before the GPU is touched
    cpu = None
    if args.config != "C5" and not args.no_cpu_baseline:
        cpu = cpu_baseline(args.config, lattices)

    import paper_1403_7560_amd as sw

    if args.copy_probe:
        copy_probe(sw, args.copy_probe)

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
        print(to_json(out), flush=True)
        return

    K = args.steps if args.steps is not None else default_steps
    W = args.warmup

    kernels = None
    if args.config == "C4":
        b = sw.Batch(lattices)
        b.sweep(W)
        t0 = time.perf_counter()
        b.sweep(K)
        dt = time.perf_counter() - t0
        b.close()
        total = sum(j["L"] ** j["dim"] for j in lattices) * K
        value = total / (dt * 1e9)
        roof = None
    else:
        value, dt, kernels, lats = timed_plain(sw, lattices, W, K, args.labeller)
        for lat in lats:
            lat.close()
        kb = kernels.get("k_bond")
        # (no k_bond launch is timed when no sweep index of the timed region
        # is a multiple of 16)
        roof = None if kb is None else {
            "bound": "hbm", "achieved": kb["achieved_GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": kb["frac"],
            "traffic": load_traffic(args.config, kb["algorithmic_bytes_per_launch"]),
            "kernel": "k_bond (bond generation + tile labelling)",
            "algorithmic_bytes_per_launch": kb["algorithmic_bytes_per_launch"],
            "avg_launch_us": kb["avg_us"]}

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
                   "sweeps_per_lattice": K,
                   "labeller": {None: "union", 0: "Hawick", 1: "Kalentev", 2: "union"}[args.labeller]},
        "roofline": roof,
        "kernels": kernels,
        "cpu_baseline": cpu,
        "job_hbm": job_hbm(sum(j["L"] ** j["dim"] * algorithmic_bytes_per_site(j["model"]) for j in lattices) * K, dt),
    }
    if args.config in PAPER_CONTEXT:
        out["paper_context"] = PAPER_CONTEXT[args.config]
    if args.config == "C2" and not args.quick:
        # the other workloads, compact (same step counts as the main line)
        # the paper's tables give "update" and "update + measurement" rows:
        # every plain leg measures each sweep; update_only is the same leg
        # with the measurement off
        out["update_only"] = dict(update_only(sw, lattices, W, K), workload="C2 pair, measurement off")
        out["c3_plain"] = dict(leg_plain(sw, inputs, "C3", W, K), workload=DESCRIPTION["C3"],
                               paper_context=PAPER_CONTEXT["C3"],
                               update_only=update_only(sw, inputs.workload("C3")[0], W, K))
        out["c4_batched"] = dict(leg_batched(sw, inputs, "C4", W, K), workload=DESCRIPTION["C4"])
        out["clock_q512"] = dict(leg_plain(sw, inputs, "CLOCK-512", W, K), workload=DESCRIPTION["CLOCK"],
                                 paper_context=PAPER_CONTEXT["CLOCK"],
                                 update_only=update_only(sw, inputs.workload("CLOCK-512")[0], W, K))
        c5 = {}
        # 300 jobs at the configured 200/s (the offered load is several times
        # what one GPU serves, so the latencies measure a growing queue), and
        # 60 jobs at 20/s, below the served rate
        for tag, n_jobs, rate in (("at_200_per_s", 300, 200.0), ("at_20_per_s", 60, 20.0)):
            r = served(n_jobs, rate, plain=(tag == "at_200_per_s"))
            c5[tag] = {"value": round(r["value"], 3), "jobs": n_jobs, "rate_per_s": rate,
                       "latency_s": r["latency_s"], "offered_load": r["offered_load"],
                       "offered_over_served": r["offered_over_served"], "job_hbm": r["job_hbm"]}
            if r["plain_form"]:
                c5[tag]["plain_form"] = r["plain_form"]
                c5[tag]["speedup_vs_plain"] = r["speedup_vs_plain"]
        out["c5_served"] = dict(c5, workload=DESCRIPTION["C5"])
    print(to_json(out), flush=True)


if __name__ == "__main__":
    main()
