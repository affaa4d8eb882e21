"""Benchmark: Metropolis trial moves per second of the treecode path on one MI355X.

A step is one pass of the whole path over one synthetic system: build the
octree with images, keys, sort, moments (from the same initial positions every
step), then run the system's trial moves with the treecode energy change,
Metropolis test and local commit, all on the device.

Headline workload: the spherical colloid (a = 10, Q = -50, eps 2/80), N = 10^4
monovalent ions plus one Kelvin image each, 10^5 trial moves per step, at the
(theta, p, N_0) that the tuner picked as the fastest setting meeting a relative
error of 1e-4 against the direct sum on both measures (eq. 4.1 and the total
energy); the accuracy is measured again here at the start and at the end of
the run.  Further legs: the same system at the stated theta = 0.5, p = 6; the
256 uneven replicas (one persistent launch per sweep under a hipGraph) and one
of them run alone as a plain chain; the 64 replicas of 199,999 ions (p = 8)
with the energy gradient after each sweep and one run alone; the 10^5-ion
gradient; the roofline of the dominant kernel against the measured copy
bandwidth; and the CPU oracle timed on the host on bounded samples.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-batched] [--no-large] [--no-cpu]
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
CU_L2_GBS = 64 * 2.4  # one CU's L2 read path: 64 B per clock at 2.4 GHz

# Settings picked by `python -m paper_1305_1825_amd.tune` on one MI355X (fastest meeting
# E(4.1) <= 1e-4 and |E - E_dir| / |E_dir| <= 1e-4); the bench measures both errors again.
GATED_CHAIN = dict(theta=0.4, p=5, n0=0)
GATED_REPLICAS = dict(theta=0.3, p=5, n0=0)

# HBM bytes per dispatch from the FETCH_SIZE / WRITE_SIZE counter passes (scaled by the same
# counters on a plain device copy), valid only for the sources they were taken on.
MEASURED_TRAFFIC = {
    "csrc": "33b3ffaf2752",
    "chain": {"units": 100000, "bytes": 183182607},        # eval_p5::k_mcb<512>, 10^5 moves
    "sweep": {"units": 3038540, "bytes": 1.02800e12},      # eval_p5::k_mcb<512>, one sweep of 256 replicas
    "sweep_fp32": {"units": 3038540, "bytes": 5.87033e11}, # the same with the single-precision far field
    "grad": {"units": 1, "bytes": 3.16016e9},              # eval_p6::k_grad, one call at 10^5 ions
}


def csrc_hash() -> str:
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_1305_1825_amd", "csrc")
    for f in sorted(os.listdir(d)):
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:12]


def traffic(kind, units):
    """Measured HBM bytes of one launch over `units` trial moves (or calls), or None when the
    sources changed since the counters were taken or the launch size differs."""
    t = MEASURED_TRAFFIC
    if t.get("csrc") != csrc_hash() or kind not in t or t[kind]["units"] != units:
        return None
    return t[kind]["bytes"]


def kernel_label(tune, p):
    """The Metropolis kernel an autotuned handle launches: one trial move per traversal (k_mc)
    or rounds of several (k_mcb), 512- or 256-thread workgroups."""
    mpr = tune.get("moves_per_round", 1)
    width = 512 if tune.get("shape_index", 0) == 0 else 256
    name = "k_mc<%d, false>" % width if mpr == 1 else "k_mcb<%d>" % width
    return "%s (p=%d, %s, %d trial move%s per traversal)" % (name, p, tune.get("shape", ""), mpr, "" if mpr == 1 else "s")


def log(*a):
    print("bench:", *a, file=sys.stderr, flush=True)


# ---------------------------------------------------------------- algorithmic bytes
def algorithmic_bytes_per_move(c, n_sample=400, replica=0, accept=0.9):
    """Bytes a move must touch at least, from the oracle's interaction counts:
    48 B per visited cell (centre and half side, 32 B; count, link, leaf slot
    base and capacity, 16 B), 8 B per moment of every far cell, 32 B per near
    source (x, y, z, q), and for an accepted move a read and a write of every
    moment on the root paths."""
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
    per_eval = (48.0 * tot_v + 8.0 * nterms * tot_f + 32.0 * tot_s) / max(evald, 1)
    frac_eval = evald / n_sample
    depth = inf["depth"] + 1
    paths = 4 if P["images"] else 2
    commit = paths * depth * nterms * 16.0
    return dict(per_move=per_eval * frac_eval + commit * accept,
                per_eval=per_eval, visited=tot_v / max(evald, 1), far=tot_f / max(evald, 1),
                near=tot_s / max(evald, 1), eval_fraction=frac_eval, commit_bytes=commit)


def batched_bytes_per_move(params, R=256, seed=0, sample=8, moves=150):
    """Algorithmic bytes per trial move of the replica workload: the same count as for
    the chain on a sample of replicas spread over the size range, weighted by N_r (a sweep
    makes N_r moves of replica r)."""
    from paper_1305_1825_amd import workloads as W
    sizes = [int(v) for v in W.replica_sizes(R, seed=seed)]
    order = sorted(range(R), key=lambda r: sizes[r])
    pick = [order[int(k * (R - 1) / (sample - 1))] for k in range(sample)]
    tot_b = tot_n = 0.0
    for r in pick:
        P, x, y, z, q = W.batched_replica(r, sizes[r], seed=seed)
        c = dict(params=dict(P, **params), x=x, y=y, z=z, q=q, seed=seed, step=1.0)
        ab = algorithmic_bytes_per_move(c, n_sample=moves, replica=r)
        tot_b += ab["per_move"] * sizes[r]
        tot_n += sizes[r]
    return tot_b / tot_n


# ---------------------------------------------------------------- GPU legs
def copy_probe(mib=2048, reps=10):
    """Achievable HBM bandwidth: a plain device-to-device copy, read + write bytes / time."""
    import torch
    src = torch.ones(mib << 17, dtype=torch.float64, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(s)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2.0 * src.numel() * 8 / (ms / 1000.0) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return dict(gbs=gbs, bytes_per_copy=2 * (mib << 20), ms_per_copy=ms)


def run_plain(c, steps, warmup, tune=True, moves_per_round=0):
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
        nonlocal last, final
        t = bhmc.Tree(P, x, y, z, q)
        if tune and "choice" not in shape:  # the first step picks shape and tile, later steps reuse them
            shape.update(t.autotune(seed=c["seed"], step=c["step"], trial_moves=1000))
        elif "choice" in shape:
            t.set_shape(shape["shape_index"])
            t.set_moves_per_round(shape["moves_per_round"])
        else:
            shape["moves_per_round"] = t.set_moves_per_round(moves_per_round)
        ev0 = torch.cuda.Event(enable_timing=True)
        ev1 = torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        st = t.mc_run(seed=c["seed"], n_moves=moves, step=c["step"])
        ev1.record(stream)
        ev1.synchronize()
        if timed:
            mc_ms.append(ev0.elapsed_time(ev1))
        last = st
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


def chain_kernel_rate(P, x, y, z, q, moves, seed=0, step=1.0, replica=0, moves_per_round=1):
    """One chain alone (512 threads on one CU), trial moves per second of kernel time;
    moves_per_round = 1 is the plain single-chain kernel (one move at a time)."""
    import torch
    from paper_1305_1825_amd import bhmc
    t = bhmc.Tree(P, x, y, z, q)
    t.set_moves_per_round(moves_per_round)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    st = t.mc_run(seed=seed, n_moves=moves, step=step, replica=replica)
    e1.record(s)
    e1.synchronize()
    t.close()
    return dict(moves=moves, ms=e0.elapsed_time(e1), moves_per_s=moves / (e0.elapsed_time(e1) / 1000.0),
                accepted=st["accepted"])


def accuracy(P, x, y, z, q):
    """The paper's error measure E of eq. 4.1, sqrt(sum (V_i - V~_i)^2 / sum V_i^2) with
    V_i = q_i phi_i, and |E_tree - E_dir| / |E_dir|.  The direct sum is the same library at
    theta = 0 (every cell opened)."""
    from paper_1305_1825_amd import bhmc
    t = bhmc.Tree(P, x, y, z, q)
    E_tree, phi_t = t.energy(with_phi=True)
    t.close()
    d = bhmc.Tree(dict(P, theta=0.0, n0=0), x, y, z, q)
    E_dir, phi_d = d.energy(with_phi=True)
    d.close()
    V, Vt = q * phi_d.cpu().numpy(), q * phi_t.cpu().numpy()
    e41 = float(np.sqrt(np.sum((V - Vt) ** 2) / np.sum(V ** 2)))
    erel = abs(E_tree - E_dir) / abs(E_dir)
    return {"E_4_1": e41, "E_rel": erel, "E_tree": E_tree, "E_direct": E_dir, "meets_1e-4": max(e41, erel) <= 1e-4}


def run_lines(c, moves, M=4, p=6, calls=5):
    """The headline system with M line images per ion besides each Kelvin image, at order p
    (the headline's theta): the chain one move per traversal (kernel time) beside the same
    chain with the Kelvin image alone, the energy and the energy with its gradient, and the
    accuracy of both ends of the chain against the same model summed directly."""
    import torch
    from paper_1305_1825_amd import bhmc
    P = dict(c["params"], line_images=M, p=p)
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    ch = chain_kernel_rate(P, x, y, z, q, moves=moves, seed=c["seed"], step=c["step"])
    ck = chain_kernel_rate(dict(P, line_images=0), x, y, z, q, moves=moves, seed=c["seed"], step=c["step"])
    t = bhmc.Tree(P, x, y, z, q)
    t.energy()
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(calls):
        t.energy()
    e1.record(s)
    e1.synchronize()
    energy_ms = e0.elapsed_time(e1) / calls
    t.energy_grad()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(calls):
        t.energy_grad()
    e1.record(s)
    e1.synchronize()
    grad_ms = e0.elapsed_time(e1) / calls
    t.mc_run(seed=c["seed"], n_moves=moves, step=c["step"])
    fx, fy, fz, fq = (v.cpu().numpy() for v in t.state())
    t.close()
    a0, a1 = accuracy(P, x, y, z, q), accuracy(P, fx, fy, fz, fq)
    return {"workload": "as the headline at p=%d, plus %d line-image sources per ion "
                        "(sigma = eps_out/(eps_in+eps_out))" % (p, M),
            "sources": (2 + M) * len(x), "chain_moves_per_s": ch["moves_per_s"], "chain_moves": moves,
            "chain_accepted": ch["accepted"],
            "kernel": "eval_p%d::k_mc<512, true> (the move kernel with the line-image steps, one move per "
                      "traversal)" % p,
            "kelvin_only_chain_moves_per_s": ck["moves_per_s"],
            "energy_ms": energy_ms, "energy_and_gradient_ms": grad_ms,
            "accuracy_start": {k: a0[k] for k in ("E_4_1", "E_rel", "meets_1e-4")},
            "accuracy_end": {k: a1[k] for k in ("E_4_1", "E_rel", "meets_1e-4")}}


def timed_sweeps(R, sweeps, params, seed=0):
    """One autotuned handle of the R replicas: a warm-up sweep (which builds the graph),
    then `sweeps` timed sweeps; and the accuracy on the smallest, median and largest replica."""
    import torch
    from paper_1305_1825_amd import bhmc, workloads as W
    sizes = [int(v) for v in W.replica_sizes(R, seed=seed)]
    reps = [W.batched_replica(r, n, seed=seed) for r, n in enumerate(sizes)]
    Ps = [dict(rp[0], **params) for rp in reps]
    cat = [torch.as_tensor(np.concatenate([rp[k] for rp in reps]), dtype=torch.float64, device="cuda:0")
           for k in range(1, 5)]
    t = bhmc.Tree(Ps, *cat, n_per_replica=sizes)
    tune = t.autotune(seed=seed, step=1.0, trial_moves=2000)
    t.batch_sweep(seed=seed, n_sweeps=1, step=1.0, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = t.batch_sweep(seed=seed, n_sweeps=sweeps, step=1.0, use_graph=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    moves = sum(s["moves"] for s in st)
    rebuilds = sum(s["rebuilds"] for s in st)
    t.close()
    # accuracy on replicas spread over the size range, at their built positions
    order = sorted(range(R), key=lambda r: sizes[r])
    acc = []
    for r in (order[0], order[R // 2], order[-1]):
        P, x, y, z, q = reps[r]
        a = accuracy(Ps[r], x, y, z, q)
        acc.append(dict(replica=r, n=sizes[r], **{k: a[k] for k in ("E_4_1", "E_rel", "meets_1e-4")}))
    return dict(moves=moves, wall=wall, rebuilds=rebuilds, autotune=tune, accuracy=acc, sizes=sizes, reps=reps, Ps=Ps,
                order=order)


def run_batched(R, sweeps, params, seed=0, far32=True):
    sw = timed_sweeps(R, sweeps, params, seed)
    moves, wall, rebuilds, tune, acc = sw["moves"], sw["wall"], sw["rebuilds"], sw["autotune"], sw["accuracy"]
    sizes, reps, Ps, order = sw["sizes"], sw["reps"], sw["Ps"], sw["order"]
    # the plain single-chain kernel on one median replica, same parameters, as many moves as one
    # of its sweeps
    rm = order[R // 2]
    P, x, y, z, q = reps[rm]
    plain = chain_kernel_rate(Ps[rm], x, y, z, q, moves=sizes[rm], seed=seed, replica=0)
    rounds = chain_kernel_rate(Ps[rm], x, y, z, q, moves=sizes[rm], seed=seed, replica=0, moves_per_round=0)
    out = dict(moves=moves, wall=wall, moves_per_s=moves / wall, replicas=R, sweeps=sweeps, rebuilds=rebuilds,
               n_min=min(sizes), n_max=max(sizes), n_total=sum(sizes), autotune=tune, params=params,
               accuracy=acc, plain_median_replica=dict(replica=rm, n=sizes[rm], **plain),
               rounds_median_replica=dict(replica=rm, n=sizes[rm], **rounds),
               ratio_vs_plain=(moves / wall) / plain["moves_per_s"])
    if far32:
        # the same sweeps with the single-precision far field (FP64 sums), gated the same way
        f = timed_sweeps(R, sweeps, dict(params, far_fp32=1), seed)
        out["far_fp32"] = dict(moves_per_s=f["moves"] / f["wall"], moves=f["moves"], wall=f["wall"],
                               autotune=f["autotune"], accuracy=f["accuracy"],
                               gate_met=all(a["meets_1e-4"] for a in f["accuracy"]),
                               traffic=traffic("sweep_fp32", f["moves"] // sweeps))
    return out


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
    # the tree built again from the same positions (what the autograd backward pays first)
    b0 = torch.cuda.Event(enable_timing=True)
    b1 = torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    t.rebuild()
    b1.record(stream)
    b1.synchronize()
    inf = t.info()
    t.close()
    med = float(np.median(ms))
    tr = traffic("grad", 1)
    return dict(workload="N=100000 ions + images, shell 10.5<r<120, theta=%.1f, p=6, leaf 16" % theta,
                ms_per_gradient=med, ms_energy_only=e0.elapsed_time(e1), ratio_to_energy=med / e0.elapsed_time(e1),
                ms_build=b0.elapsed_time(b1),
                ions_per_s=len(c["x"]) / (med / 1000.0), E=E, ncell=inf["ncell"],
                traffic=tr,
                # measured HBM bytes of k_grad over the whole call's time: far below the 8 TB/s
                # peak, the kernel is bound by its FP64 evaluation of the far cells
                hbm_gbs=(tr / (med / 1000.0) / 1e9 if tr else None))


def run_large(sweeps, grad_each=True):
    """64 replicas of the 199,999-ion 2:1 electrolyte (theta = 0.5, p = 8, leaf 32): sweeps,
    each followed by the energy gradient of every replica; one replica alone through the
    plain chain kernel; accuracy of one replica against the direct sum."""
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
    tune = t.autotune(seed=0, step=1.0, trial_moves=256)
    sweep_s, grad_s, moves = [], [], 0
    for s in range(sweeps):
        t0 = time.perf_counter()
        st = t.batch_sweep(seed=0, n_sweeps=1, step=1.0, use_graph=True)
        torch.cuda.synchronize()
        sweep_s.append(time.perf_counter() - t0)
        moves += sum(v["moves"] for v in st)
        if grad_each:
            t0 = time.perf_counter()
            for r in range(R):
                t.energy_grad(replica=r)
            torch.cuda.synchronize()
            grad_s.append(time.perf_counter() - t0)
        log("large: sweep %d of %d done" % (s + 1, sweeps))
    t.close()
    wall = sum(sweep_s)
    c0 = reps[0]
    plain = chain_kernel_rate(c0["params"], c0["x"], c0["y"], c0["z"], c0["q"], moves=20000)
    rounds = chain_kernel_rate(c0["params"], c0["x"], c0["y"], c0["z"], c0["q"], moves=20000, moves_per_round=0)
    acc = accuracy(c0["params"], c0["x"], c0["y"], c0["z"], c0["q"])
    return dict(workload="64 replicas x N=199999 (2:1, a=20, Q=-200, shell 20.5<r<200) + images, "
                         "theta=0.5, p=8, leaf 32", replicas=R, sweeps=sweeps, moves=moves,
                wall=wall, moves_per_s=moves / wall, build_s=build_s, autotune=tune,
                gradient_s_per_sweep=(float(np.mean(grad_s)) if grad_s else None),
                gradient_ms_per_replica=(1000.0 * float(np.mean(grad_s)) / R if grad_s else None),
                plain_one_replica=plain, rounds_one_replica=rounds, ratio_vs_plain=(moves / wall) / plain["moves_per_s"],
                accuracy_replica0={k: acc[k] for k in ("E_4_1", "E_rel", "meets_1e-4")})


# ---------------------------------------------------------------- CPU oracle
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
                sample="first %d trial moves of the headline chain (N=10000 colloid, serial C treecode, "
                       "build excluded), %.1f s" % (done, dt))


def cpu_direct(c, seconds=6.0):
    """The oracle's direct-sum Metropolis chain (eq. 1.1 energy change, O(N) per move) on one core."""
    import oracle as O
    x, y, z = c["x"].copy(), c["y"].copy(), c["z"].copy()
    done, chunk = 0, 200
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        r = O.direct_mc_run(c["params"], x, y, z, c["q"], c["seed"], 0, done, chunk, c["step"])
        x, y, z = r["x"], r["y"], r["z"]
        done += chunk
    dt = time.perf_counter() - t0
    return dict(value=done / dt, unit="moves/s", cores=1, kind="oracle direct sum",
                sample="first %d trial moves of the headline chain with the direct energy change, %.1f s" % (done, dt))


def _replica_worker(args):
    r, n, seconds, params = args
    import oracle as O
    from paper_1305_1825_amd import workloads as W
    P, x, y, z, q = W.batched_replica(r, n, seed=0)
    o = O.Tree(dict(P, **params), x, y, z, q)
    done, chunk = 0, 500
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and done < n:
        o.mc_run(seed=0, replica=r, move0=done, n_moves=min(chunk, n - done), step=1.0)
        done += min(chunk, n - done)
    return done, time.perf_counter() - t0


def cpu_replicas(params, seconds=8.0):
    """One replica per host core (the oracle's treecode chain of replicas 0.. of the
    256-replica workload), aggregate trial moves per second."""
    import multiprocessing as mp
    from paper_1305_1825_amd import workloads as W
    cores = max(1, min(16, os.cpu_count() or 1))
    sizes = [int(v) for v in W.replica_sizes(256, seed=0)]
    jobs = [(r, sizes[r], seconds, params) for r in range(cores)]
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        out = pool.map(_replica_worker, jobs)
    wall = time.perf_counter() - t0
    rate = sum(d / s for d, s in out)
    return dict(value=rate, unit="moves/s", cores=cores, kind="oracle, one replica per core",
                sample="replicas 0..%d of the 256-replica workload, %.0f s of chain each (wall %.1f s)"
                       % (cores - 1, seconds, wall))


# ---------------------------------------------------------------- main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--moves", type=int, default=100000)
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-sweeps", type=int, default=10)
    ap.add_argument("--no-large", action="store_true")
    ap.add_argument("--large-sweeps", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-gradient", action="store_true")
    ap.add_argument("--no-stated", action="store_true", help="skip the theta=0.5, p=6 leg")
    ap.add_argument("--no-lines", action="store_true", help="skip the multiple-image leg")
    ap.add_argument("--line-moves", type=int, default=20000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB once with a plain device copy (the reference dispatch of the "
                         "HBM counter passes)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(replicas would shard one per GPU with no exchange; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1305_1825_amd import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy << 17, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read and %d written" % (src.numel() * 8, src.numel() * 8))
        del src, dst
        torch.cuda.empty_cache()
    log("copy probe")
    probe = copy_probe()
    achievable = probe["gbs"]

    c = W.config_colloid_10k()
    c["params"] = dict(c["params"], **GATED_CHAIN)
    c["moves"] = args.moves
    log("plain chain %s at %s, %d moves/step, %d steps" % (c["name"], GATED_CHAIN, c["moves"], args.steps))
    res = run_plain(c, args.steps, args.warmup)
    total_moves = args.steps * c["moves"]
    value = total_moves / res["wall"]
    ms_per_step = 1000.0 * res["wall"] / args.steps
    mc_ms = float(np.mean(res["mc_ms"]))
    ab = algorithmic_bytes_per_move(c, accept=res["stats"]["accepted"] / max(res["stats"]["moves"], 1))
    achieved = ab["per_move"] * c["moves"] / (mc_ms / 1000.0) / 1e9
    g = GATED_CHAIN
    out = {
        "metric": "Metropolis trial moves/sec (treecode dE, 1 GPU) at <=1e-4 relative error",
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
                               "shell 10.5<r<40, hard core 0.5, theta=%.1f, p=%d, N_0=%d, leaf 16, "
                               "%d trial moves per step (build included)" % (g["theta"], g["p"], g["n0"], c["moves"]),
                   "chain": "one chain, trial moves evaluated in rounds of up to 8 and decided in order",
                   "seed": c["seed"]},
        "stats": res["stats"],
        "autotune": res["autotune"],
        "mc_kernel_ms_per_step": mc_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic("chain", c["moves"]),
                     "achievable": achievable, "frac_achievable": achieved / achievable,
                     "per_cu": {"peak": CU_L2_GBS, "frac": achieved / CU_L2_GBS,
                                "note": "one workgroup on one CU: bytes through that CU over its L2 path"},
                     "kernel": kernel_label(res["autotune"], g["p"]),
                     "algorithmic_bytes_per_move": ab["per_move"],
                     "per_move_counts": {k: ab[k] for k in ("visited", "far", "near", "eval_fraction")}},
        "copy_probe": probe,
        "csrc": csrc_hash(),
    }
    log("the headline chain one move at a time (plain single-chain kernel)")
    plain_c = chain_kernel_rate(c["params"], c["x"], c["y"], c["z"], c["q"], moves=c["moves"], seed=c["seed"])
    out["plain_single_move_chain"] = plain_c
    out["rounds_vs_single_move"] = (c["moves"] / (mc_ms / 1000.0)) / plain_c["moves_per_s"]
    log("accuracy of the headline against the direct sum")
    acc = {"start": accuracy(c["params"], c["x"], c["y"], c["z"], c["q"])}
    fx, fy, fz, fq = res["final"]
    acc["end"] = accuracy(c["params"], fx, fy, fz, fq)
    acc["gate"] = "E(4.1) and |E - E_dir|/|E_dir| both <= 1e-4 at the start and the end"
    acc["gate_met"] = all(acc[k]["meets_1e-4"] for k in ("start", "end"))
    out["accuracy"] = acc
    if not args.no_stated:
        log("the stated theta=0.5, p=6 chain")
        cs = W.config_colloid_10k()
        rs = run_plain(cs, 1, 0, tune=False)
        out["stated_theta05_p6"] = {"moves_per_s": cs["moves"] / (rs["mc_ms"][0] / 1000.0),
                                    **{k: v for k, v in accuracy(cs["params"], cs["x"], cs["y"], cs["z"],
                                                                 cs["q"]).items() if k != "E_tree"}}
    if not args.no_stated:
        log("the headline chain with the single-precision far field")
        cf = dict(c, params=dict(c["params"], far_fp32=1))
        rf = run_plain(cf, 1, 0, tune=False)
        ff = rf["final"]
        a0, a1 = accuracy(cf["params"], c["x"], c["y"], c["z"], c["q"]), accuracy(cf["params"], *ff)
        out["far_fp32_chain"] = {
            "moves_per_s": c["moves"] / (rf["mc_ms"][0] / 1000.0),
            "note": "far cells evaluated in FP32 from an FP32 copy of the moments, every sum in FP64",
            "accuracy_start": {k: a0[k] for k in ("E_4_1", "E_rel", "meets_1e-4")},
            "accuracy_end": {k: a1[k] for k in ("E_4_1", "E_rel", "meets_1e-4")},
            "gate_met": a0["meets_1e-4"] and a1["meets_1e-4"]}
    if not args.no_lines:
        log("the headline system with the multiple-image model (M = 4 line images per ion)")
        out["line_images"] = run_lines(c, args.line_moves)
    if not args.no_batched:
        log("batched replicas")
        b = run_batched(256, args.batched_sweeps, GATED_REPLICAS)
        bpm = batched_bytes_per_move(GATED_REPLICAS)
        ach = bpm * b["moves_per_s"] / 1e9
        b["roofline"] = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBS, "achievable": achievable, "frac_achievable": ach / achievable,
                         "traffic": traffic("sweep", b["moves"] // b["sweeps"]),
                         "kernel": kernel_label(b["autotune"], GATED_REPLICAS["p"]) + ", one sweep per launch",
                         "algorithmic_bytes_per_move": bpm}
        b["ratio_vs_headline_chain"] = b["moves_per_s"] / value
        out["batched"] = b
    if not args.no_large:
        log("large replicas")
        out["large"] = run_large(args.large_sweeps)
    if not args.no_gradient:
        log("gradient N=1e5")
        out["gradient"] = run_gradient()
    if not args.no_cpu:
        log("cpu baselines (oracle)")
        out["cpu_baseline"] = cpu_baseline(c)
        d = cpu_direct(c)
        rep = cpu_replicas(GATED_REPLICAS)
        out["cpu_baselines"] = {
            "direct_sum_1core": d,
            "replicas_all_cores": rep,
            "oracle_tree_vs_direct": out["cpu_baseline"]["value"] / d["value"],
            "paper_context": "the paper reports about 100x for its treecode over direct summation at N ~ 1e4 "
                             "(serial, 2.67 GHz CPU); the ratio above is the oracle's on this host",
        }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
