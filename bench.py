"""Benchmark: Metropolis trial moves per second of the treecode path on one MI355X.

A step is one pass of the whole path over one synthetic system: build the
octree with images, keys, sort, moments (from the same initial positions every
step), then run the system's trial moves with the treecode energy change,
Metropolis test and local commit, all on the device.

Headline workload: spherical colloid, N = 10,000 monovalent ions plus one
Kelvin image each, theta = 0.5, p = 6, leaf 16, 100,000 trial moves per step.
Extra objects: the batched-replica workload (256 replicas of uneven N, one
persistent launch per sweep under a hipGraph) and the roofline of the dominant
kernel, plus the CPU oracle timed on the host on a bounded sample.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batched] [--no-cpu]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per dispatch from the FETCH_SIZE / WRITE_SIZE counter passes (scaled by the same
# counters on a plain 256 MiB device copy), valid only for the sources they were taken on.
MEASURED_TRAFFIC = {
    "csrc": "39c0901e87ab",
    "chain": {"moves": 100000, "bytes": 347086782, "l2_hit_rate": 0.9976},
    "sweep": {"moves": 3038540, "bytes": 307839059374, "l2_hit_rate": 0.5779},
}


def csrc_hash() -> str:
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_1305_1825_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:12]


def traffic(kind, moves):
    """Measured HBM bytes of one launch of `moves` trial moves, or None when the
    sources changed since the counters were taken or the launch size differs."""
    t = MEASURED_TRAFFIC
    if t["csrc"] != csrc_hash() or t[kind]["moves"] != moves:
        return None
    return t[kind]["bytes"]


def algorithmic_bytes_per_move(c, n_sample=400, replica=0):
    """Bytes a move must touch at least, from the oracle's interaction counts:
    40 B per visited cell (centre, half side, count, link), 8 B per moment of
    every far cell, 32 B per near source (x, y, z, q), and for an accepted move
    a read and a write of every moment on the four root paths."""
    import oracle as O
    P = c["params"]
    o = O.Tree(P, c["x"], c["y"], c["z"], c["q"])
    inf = o.info()
    nterms = inf["nterms"]
    n = len(c["x"])
    tot_v = tot_f = tot_s = 0
    evald = 0
    for m in range(n_sample):
        i, d, _ = O.draw_move(c["seed"], replica, m, n, c["step"])
        rn = np.array([c["x"][i], c["y"][i], c["z"][i]]) + d
        _, reason, cnt = o.delta(i, rn, counts=True)
        if reason == 0:
            tot_v += cnt[0]; tot_f += cnt[1]; tot_s += cnt[2]
            evald += 1
    per_eval = (40.0 * tot_v + 8.0 * nterms * tot_f + 32.0 * tot_s) / max(evald, 1)
    frac_eval = evald / n_sample
    depth = inf["depth"] + 1
    paths = 4 if P["images"] else 2
    commit = paths * depth * nterms * 16.0
    return dict(per_move=per_eval * frac_eval + commit * 0.9 * frac_eval,
                per_eval=per_eval, visited=tot_v / max(evald, 1), far=tot_f / max(evald, 1),
                near=tot_s / max(evald, 1), eval_fraction=frac_eval, commit_bytes=commit)


def run_plain(c, steps, warmup, tune=True):
    import torch
    from paper_1305_1825_amd import bhmc
    P = c["params"]
    x, y, z, q = (torch.as_tensor(a, dtype=torch.float64, device="cuda:0") for a in (c["x"], c["y"], c["z"], c["q"]))
    moves = c["moves"]
    stream = torch.cuda.current_stream()
    mc_ms = []
    last = None
    final = None

    shape = {}

    def one_step(timed):
        nonlocal last
        t = bhmc.Tree(P, x, y, z, q)
        if tune and not shape:  # the warm-up step picks the launch shape, later steps reuse it
            shape.update(t.autotune(seed=c["seed"], step=c["step"], trial_moves=1000))
        elif shape:
            t.set_shape(shape["choice"])
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        st = t.mc_run(seed=c["seed"], n_moves=moves, step=c["step"])
        ev1.record(stream)
        ev1.synchronize()
        if timed:
            mc_ms.append(ev0.elapsed_time(ev1))
        last = st
        nonlocal final
        final = [v.cpu().numpy() for v in t.state()]
        t.close()

    for _ in range(warmup):
        one_step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(wall=wall, mc_ms=mc_ms, stats=last, final=final, autotune=shape)


def batched_bytes_per_move(R=256, seed=0, sample=8, moves=150):
    """Algorithmic bytes per trial move of the replica workload: the same count as
    for the chain on a sample of replicas spread over the size range, weighted by N_r
    (a sweep makes N_r moves of replica r)."""
    from paper_1305_1825_amd import workloads as W
    sizes = [int(v) for v in W.replica_sizes(R, seed=seed)]
    order = sorted(range(R), key=lambda r: sizes[r])
    pick = [order[int(k * (R - 1) / (sample - 1))] for k in range(sample)]
    tot_b = tot_n = 0.0
    for r in pick:
        P, x, y, z, q = W.batched_replica(r, sizes[r], seed=seed)
        c = dict(params=P, x=x, y=y, z=z, q=q, seed=seed, step=1.0)
        ab = algorithmic_bytes_per_move(c, n_sample=moves, replica=r)
        tot_b += ab["per_move"] * sizes[r]
        tot_n += sizes[r]
    return tot_b / tot_n


def run_batched(R, sweeps, seed=0):
    import torch
    from paper_1305_1825_amd import bhmc, workloads as W
    sizes = [int(v) for v in W.replica_sizes(R, seed=seed)]
    reps = [W.batched_replica(r, n, seed=seed) for r, n in enumerate(sizes)]
    Ps = [rp[0] for rp in reps]
    cat = [torch.as_tensor(np.concatenate([rp[k] for rp in reps]), dtype=torch.float64, device="cuda:0")
           for k in range(1, 5)]
    t = bhmc.Tree(Ps, *cat, n_per_replica=sizes)
    tune = t.autotune(seed=seed, step=1.0, trial_moves=2000)
    t.batch_sweep(seed=seed, n_sweeps=1, step=1.0, use_graph=True)  # warm-up sweep, builds the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = t.batch_sweep(seed=seed, n_sweeps=sweeps, step=1.0, use_graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    moves = sum(s["moves"] for s in st)
    rebuilds = sum(s["rebuilds"] for s in st)
    t.close()
    return dict(moves=moves, wall=wall, moves_per_s=moves / wall, replicas=R, sweeps=sweeps, rebuilds=rebuilds,
                n_min=min(sizes), n_max=max(sizes), n_total=sum(sizes), autotune=tune)


def run_gradient(theta=0.5, calls=3):
    """Energy plus exact gradient of the 1e5-ion shell system, inputs resident."""
    import torch
    from paper_1305_1825_amd import bhmc, workloads as W
    c = W.config_gradient_100k(theta=theta)
    x, y, z, q = (torch.as_tensor(c[k], dtype=torch.float64, device="cuda:0") for k in ("x", "y", "z", "q"))
    t = bhmc.Tree(c["params"], x, y, z, q)
    t.energy_grad()  # allocates the workspace
    stream = torch.cuda.current_stream()
    ms = []
    for _ in range(calls):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        E, g, gq = t.energy_grad()
        e1.record(stream)
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t.energy()
    e1.record(stream)
    e1.synchronize()
    inf = t.info()
    t.close()
    return dict(workload="N=100000 ions + images, shell 10.5<r<120, theta=%.1f, p=6, leaf 16" % theta,
                ms_per_gradient=float(np.median(ms)), ms_energy_only=e0.elapsed_time(e1),
                ions_per_s=len(c["x"]) / (float(np.median(ms)) / 1000.0), E=E, ncell=inf["ncell"])


def run_large(sweeps, grad_replicas):
    """64 replicas of the 199,999-ion 2:1 electrolyte (p = 8, leaf 32): sweeps, then the
    energy gradient of the first grad_replicas replicas."""
    import torch
    from paper_1305_1825_amd import bhmc, workloads as W
    R = 64
    reps = [W.config_large_asym(r=r) for r in range(R)]
    sizes = [len(rp["x"]) for rp in reps]
    cat = [torch.as_tensor(np.concatenate([rp[k] for rp in reps]), dtype=torch.float64, device="cuda:0")
           for k in ("x", "y", "z", "q")]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t = bhmc.Tree([rp["params"] for rp in reps], *cat, n_per_replica=sizes)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    tune = t.autotune(seed=0, step=1.0, trial_moves=128)
    t0 = time.perf_counter()
    st = t.batch_sweep(seed=0, n_sweeps=sweeps, step=1.0, use_graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    moves = sum(s["moves"] for s in st)
    t0 = time.perf_counter()
    for r in range(grad_replicas):
        t.energy_grad(replica=r)
    torch.cuda.synchronize()
    gwall = time.perf_counter() - t0
    t.close()
    return dict(workload="64 replicas x N=199999 (2:1, a=20, Q=-200, shell 20.5<r<200) + images, "
                         "theta=0.5, p=8, leaf 32", replicas=R, sweeps=sweeps, moves=moves,
                wall=wall, moves_per_s=moves / wall, build_s=build_s, autotune=tune,
                gradient_s_per_replica=gwall / max(grad_replicas, 1))


def accuracy(P, x, y, z, q):
    """The paper's error measure E of eq. 4.1, sqrt(sum (V_i - V~_i)^2 / sum V_i^2) with
    V_i = q_i phi_i, and |E_tree - E_dir| / |E_dir|.  The direct sum is the same library at
    theta = 0 (every cell opened), read from dE/dq_i = l_B phi_i + the exact self-image and
    central terms."""
    from paper_1305_1825_amd import bhmc
    t = bhmc.Tree(P, x, y, z, q)
    E_tree, phi_t = t.energy(with_phi=True)
    t.close()
    d = bhmc.Tree(dict(P, theta=0.0), x, y, z, q)
    E_dir, _, dq = d.energy_grad()
    d.close()
    dq = dq.cpu().numpy()
    phi_t = phi_t.cpu().numpy()
    l, a = P["l_B"], P.get("a", 0.0)
    r2 = x * x + y * y + z * z
    extra = np.zeros_like(q)
    if P.get("geom", 0) == 1:
        if P.get("images", 0):
            gam = (P["eps_out"] - P["eps_in"]) / (P["eps_out"] + P["eps_in"])
            extra += l * gam * a * q / (r2 - a * a)
        extra += l * P.get("Q_center", 0.0) / np.sqrt(r2)
    phi_d = (dq - extra) / l
    V, Vt = q * phi_d, q * phi_t
    return {"E_4_1": float(np.sqrt(np.sum((V - Vt) ** 2) / np.sum(V ** 2))),
            "E_rel": abs(E_tree - E_dir) / abs(E_dir), "E_tree": E_tree, "E_direct": E_dir}


def cpu_baseline(c, seconds=12.0):
    import oracle as O
    P = c["params"]
    o = O.Tree(P, c["x"], c["y"], c["z"], c["q"])
    chunk = 500
    done = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < c["moves"]:
        o.mc_run(seed=c["seed"], replica=0, move0=done, n_moves=chunk, step=c["step"])
        done += chunk
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="moves/s", cores=1, kind="oracle",
                sample="first %d trial moves of the N=10000 colloid chain (serial C treecode, "
                       "build excluded), %.1f s" % (done, dt))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--moves", type=int, default=100000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-sweeps", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gradient", action="store_true")
    ap.add_argument("--large-sweeps", type=int, default=0,
                    help="also run the 64 x 199,999-ion replicas for this many sweeps")
    ap.add_argument("--large-grad", type=int, default=4, help="replicas whose gradient the large leg times")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MiB",
                    help="first copy a buffer of this size once (reference kernel for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(replicas would shard one per GPU with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1305_1825_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy << 17, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print("bench: copied %d MiB (%d bytes read, %d written)" % (args.calibrate_copy, src.numel() * 8,
                                                                    src.numel() * 8), file=sys.stderr, flush=True)
        del src, dst
    c = W.config_colloid_10k()
    c["moves"] = args.moves
    print("bench: plain chain %s, %d moves/step, %d steps" % (c["name"], c["moves"], args.steps),
          file=sys.stderr, flush=True)
    res = run_plain(c, args.steps, args.warmup)
    total_moves = args.steps * c["moves"]
    value = total_moves / res["wall"]
    ms_per_step = 1000.0 * res["wall"] / args.steps
    mc_ms = float(np.mean(res["mc_ms"]))
    ab = algorithmic_bytes_per_move(c)
    achieved = ab["per_move"] * c["moves"] / (mc_ms / 1000.0) / 1e9
    out = {
        "metric": "Metropolis trial moves/sec (treecode dE, 1 GPU)",
        "value": value,
        "unit": "moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "colloid a=10 Q=-50 eps 2/80, N=10000 ions + 10000 Kelvin images, "
                               "shell 10.5<r<40, hard core 0.5, theta=0.5, p=6, leaf 16, "
                               "%d trial moves per step (build included)" % c["moves"],
                   "chain": "plain single chain", "seed": c["seed"]},
        "stats": res["stats"],
        "autotune": res["autotune"],
        "mc_kernel_ms_per_step": mc_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic("chain", c["moves"]),
                     "kernel": "k_mc (p=6)", "algorithmic_bytes_per_move": ab["per_move"],
                     "per_move_counts": {k: ab[k] for k in ("visited", "far", "near", "eval_fraction")}},
        "csrc": csrc_hash(),
    }
    if not args.no_batched:
        print("bench: batched replicas", file=sys.stderr, flush=True)
        b = run_batched(256, args.batched_sweeps)
        b["ratio_vs_plain"] = b["moves_per_s"] / value
        bpm = batched_bytes_per_move()
        ach = bpm * b["moves_per_s"] / 1e9
        b["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "traffic": traffic("sweep", b["moves"] // b["sweeps"]),
                         "kernel": "k_mc (p=4), one sweep per launch",
                         "algorithmic_bytes_per_move": bpm}
        out["batched"] = b
    print("bench: accuracy against the direct sum", file=sys.stderr, flush=True)
    acc = {"start": accuracy(c["params"], c["x"], c["y"], c["z"], c["q"])}
    if res["final"] is not None:
        fx, fy, fz, fq = res["final"]
        acc["end"] = accuracy(c["params"], fx, fy, fz, fq)
    # the smallest p at which this workload meets E <= 1e-4, timed the same way on a shorter chain
    c7 = W.config_colloid_10k(p=7)
    c7["moves"] = 20000
    r7 = run_plain(c7, 1, 0)
    acc["at_1e-4"] = {"p": 7, "moves_per_s": c7["moves"] / (float(np.mean(r7["mc_ms"])) / 1000.0),
                      "moves": c7["moves"], **accuracy(c7["params"], c7["x"], c7["y"], c7["z"], c7["q"])}
    out["accuracy"] = acc
    if not args.no_gradient:
        print("bench: gradient N=1e5", file=sys.stderr, flush=True)
        out["gradient"] = run_gradient()
    if args.large_sweeps > 0:
        print("bench: large replicas", file=sys.stderr, flush=True)
        out["large"] = run_large(args.large_sweeps, args.large_grad)
    if not args.no_cpu:
        print("bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(c)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
