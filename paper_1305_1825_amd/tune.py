"""Opening angle, expansion order and minimum expansion number at a fixed
accuracy, picked by measurement.

The paper leaves theta, p and N_0 to the user: Sec. 3.2 defines N_0 as the
smallest cell population worth an expansion (smaller cells are summed
directly), and Sec. 4 tunes it per p by timing.  Here every candidate is
scored on one system by two errors against the direct sum (the library at
theta = 0): the measure E of eq. 4.1 over the per-ion energies, and the
relative error of the total energy.  For each theta the smallest p meeting
the target on both is kept; for it, N_0 is swept and each setting that still
meets the target is timed on a Metropolis chain on the GPU.  The fastest
candidate wins.

For the replica workload (--workload replicas) every candidate must meet the
target on the smallest, the median and the largest replica, and is timed on
whole sweeps of all 256 replicas (one persistent launch each, launch shape and
traversal tile autotuned), since a sweep loads the memory system as one chain
does not.

    python -m paper_1305_1825_amd.tune [--workload colloid|replica|replicas] [--target 1e-4] [--moves 10000]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import bhmc
from . import workloads as W


def direct_energies(P, x, y, z, q):
    """Per-ion potentials and the total energy of the direct sum (theta = 0)."""
    t = bhmc.Tree(dict(P, theta=0.0, n0=0), x, y, z, q)
    E, phi = t.energy(with_phi=True)
    t.close()
    return phi.cpu().numpy(), E


def errors(P, x, y, z, q, phi_d, E_d):
    """(E of eq. 4.1, |E_tree - E_dir| / |E_dir|) of the treecode with parameters P."""
    t = bhmc.Tree(P, x, y, z, q)
    E, phi = t.energy(with_phi=True)
    t.close()
    V, Vt = q * phi_d, q * phi.cpu().numpy()
    return float(np.sqrt(np.sum((V - Vt) ** 2) / np.sum(V ** 2))), abs(E - E_d) / abs(E_d)


def chain_rate(P, x, y, z, q, moves, step, seed=0):
    """Trial moves per second of one chain on the device (kernel time only)."""
    import torch
    t = bhmc.Tree(P, x, y, z, q)
    t.mc_run(seed=seed + 1, n_moves=min(500, moves), step=step)  # warm the kernel
    t.close()
    t = bhmc.Tree(P, x, y, z, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t.mc_run(seed=seed, n_moves=moves, step=step)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t.close()
    return moves / dt


def tune(P, x, y, z, q, target=1e-4, thetas=(0.3, 0.4, 0.5, 0.6), ps=range(2, 11),
         n0s=(0, 4, 8, 16, 32, 64), moves=10000, step=1.0, log=print):
    phi_d, E_d = direct_energies(P, x, y, z, q)
    rows = []
    for theta in thetas:
        for p in ps:
            Pc = dict(P, theta=theta, p=p, n0=0)
            e41, erel = errors(Pc, x, y, z, q, phi_d, E_d)
            if max(e41, erel) > target:
                row = {"theta": theta, "p": p, "n0": 0, "E_4_1": e41, "E_rel": erel}
                rows.append(row)
                log(json.dumps(row))
                continue
            # the smallest p meeting the target at this theta: sweep N_0
            for n0 in n0s:
                Pn = dict(Pc, n0=n0)
                if n0:
                    e41, erel = errors(Pn, x, y, z, q, phi_d, E_d)
                row = {"theta": theta, "p": p, "n0": n0, "E_4_1": e41, "E_rel": erel}
                if max(e41, erel) <= target:
                    row["moves_per_s"] = chain_rate(Pn, x, y, z, q, moves, step)
                rows.append(row)
                log(json.dumps(row))
            break
    ok = [r for r in rows if "moves_per_s" in r]
    best = max(ok, key=lambda r: r["moves_per_s"]) if ok else None
    return best, rows


def sweep_rate(params, sweeps=2, R=256, seed=0):
    """Trial moves per second of whole sweeps of the R replicas (after a warm-up sweep)."""
    import torch
    sizes = [int(v) for v in W.replica_sizes(R, seed=seed)]
    reps = [W.batched_replica(r, n, seed=seed) for r, n in enumerate(sizes)]
    cat = [torch.as_tensor(np.concatenate([rp[k] for rp in reps]), dtype=torch.float64, device="cuda:0")
           for k in range(1, 5)]
    t = bhmc.Tree([dict(rp[0], **params) for rp in reps], *cat, n_per_replica=sizes)
    tune_out = t.autotune(seed=seed, step=1.0, trial_moves=2000)
    t.batch_sweep(seed=seed, n_sweeps=1, step=1.0, use_graph=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = t.batch_sweep(seed=seed, n_sweeps=sweeps, step=1.0, use_graph=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t.close()
    return sum(v["moves"] for v in st) / dt, tune_out


def tune_replicas(target=1e-4, thetas=(0.3, 0.4, 0.5, 0.6), ps=range(3, 11), log=print):
    """(theta, p) with N_0 = 0 meeting the target on the smallest, median and largest
    replica, the smallest p per theta, timed on whole sweeps."""
    sizes = [int(v) for v in W.replica_sizes(256, seed=0)]
    order = np.argsort(sizes)
    picks = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    systems = []
    for r in picks:
        P, x, y, z, q = W.batched_replica(r, sizes[r], seed=0)
        systems.append((P, x, y, z, q) + direct_energies(P, x, y, z, q))
    rows = []
    for theta in thetas:
        for p in ps:
            errs = [errors(dict(P, theta=theta, p=p, n0=0), x, y, z, q, phi_d, E_d)
                    for P, x, y, z, q, phi_d, E_d in systems]
            e41, erel = max(e[0] for e in errs), max(e[1] for e in errs)
            row = {"theta": theta, "p": p, "n0": 0, "E_4_1": e41, "E_rel": erel}
            if max(e41, erel) <= target:
                row["moves_per_s"], row["autotune"] = sweep_rate(dict(theta=theta, p=p, n0=0))
                rows.append(row)
                log(json.dumps(row))
                break
            rows.append(row)
            log(json.dumps(row))
    ok = [r for r in rows if "moves_per_s" in r]
    return (max(ok, key=lambda r: r["moves_per_s"]) if ok else None), rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="colloid", choices=("colloid", "replica", "replicas"))
    ap.add_argument("--target", type=float, default=1e-4)
    ap.add_argument("--moves", type=int, default=10000)
    args = ap.parse_args()
    if args.workload == "replicas":
        best, _ = tune_replicas(target=args.target, log=lambda s: print(s, flush=True))
        print(json.dumps({"best": best}), flush=True)
        return
    if args.workload == "colloid":
        c = W.config_colloid_10k()
        P, x, y, z, q, step = c["params"], c["x"], c["y"], c["z"], c["q"], c["step"]
    else:  # a median-sized replica of the 256-replica workload
        sizes = [int(v) for v in W.replica_sizes(256, seed=0)]
        r = int(np.argsort(sizes)[len(sizes) // 2])
        P, x, y, z, q = W.batched_replica(r, sizes[r], seed=0)
        step = 1.0
    best, _ = tune(P, x, y, z, q, target=args.target, moves=args.moves, step=step,
                   log=lambda s: print(s, flush=True))
    print(json.dumps({"best": best}), flush=True)


if __name__ == "__main__":
    main()
