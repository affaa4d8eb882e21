"""Where the time of a batched Metropolis round goes.

Loads the instrumented library built by
    python -m paper_1305_1825_amd.build --phase-timers
(libbhmc_phase.so beside libbhmc.so; every kernel is the same, the batched
kernel's thread 0 also adds the constant-clock ticks of each phase of a round to
device counters) and reports, for one chain and for the replica sweep, the
microseconds per round and per trial move of each phase: set-up, traversal
levels, corrected moments and scan, far cells, near leaves, hard cores below far
cells, path descents, corrections, decisions, leaf index arrays and moments;
and per round the traversal's chunks of frontier entries, its entries (and how
many hold no source besides the movers'), its far and near list entries, and the
time the root-path descents and the commit prefetch take inside the level loop.

    python -m paper_1305_1825_amd.phase_profile [--moves 20000] [--no-sweep]
"""
from __future__ import annotations

import argparse
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
os.environ.setdefault("BHMC_LIB", os.path.join(HERE, "libbhmc_phase.so"))

import numpy as np  # noqa: E402

from . import bhmc  # noqa: E402
from . import workloads as W  # noqa: E402

CLOCK_HZ = 100e6  # the device's constant clock read by wall_clock64
# counters rather than ticks: level-loop chunks, frontier entries, entries with no remaining source, list entries
COUNTS = ("chunks", "entries", "empty_entries", "far_entries", "near_entries")
# ticks spent inside the traversal's level loop by the waves that also descend the root paths and
# prefetch the commit state (they overlap the level time, so they are not added to the sum)
OVERLAPPED = ("hook_paths", "hook_prefetch")


def report(name, ticks, wall_s=None):
    rounds, moves = ticks.get("rounds", 0), ticks.get("moves", 0)
    out = {"workload": name, "rounds": rounds, "moves": moves}
    if rounds:
        timed = {k: v for k, v in ticks.items() if k not in ("rounds", "moves") + COUNTS + OVERLAPPED}
        for k, v in timed.items():
            out[k + "_us_per_round"] = v / CLOCK_HZ * 1e6 / rounds
        for k in OVERLAPPED:
            if k in ticks:
                out[k + "_us_per_round_within_levels"] = ticks[k] / CLOCK_HZ * 1e6 / rounds
        out["sum_us_per_round"] = sum(timed.values()) / CLOCK_HZ * 1e6 / rounds
        for k in COUNTS:
            if k in ticks:
                out[k + "_per_round"] = ticks[k] / rounds
        if ticks.get("chunks"):
            out["levels_us_per_chunk"] = ticks["levels"] / CLOCK_HZ * 1e6 / ticks["chunks"]
        out["moves_per_round"] = moves / rounds
    if wall_s:
        out["moves_per_s"] = moves / wall_s if moves else None
    print(json.dumps(out), flush=True)
    return out


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--moves", type=int, default=20000)
    ap.add_argument("--no-sweep", action="store_true")
    args = ap.parse_args()
    c = W.config_colloid_10k()
    for th, p in ((0.4, 5), (0.5, 6)):
        P = dict(c["params"], theta=th, p=p, n0=0)
        t = bhmc.Tree(P, c["x"], c["y"], c["z"], c["q"])
        t.mc_run(seed=1, n_moves=1000, step=1.0)
        t.phase_ticks(reset=True)
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        t.mc_run(seed=0, n_moves=args.moves, step=1.0, move0=1000)
        ev1.record()
        ev1.synchronize()
        report("colloid N=1e4 chain theta=%.1f p=%d" % (th, p), t.phase_ticks(reset=True),
               ev0.elapsed_time(ev1) / 1000.0)
        t.close()
    if not args.no_sweep:
        sizes = [int(v) for v in W.replica_sizes(256, seed=0)]
        reps = [W.batched_replica(r, n, seed=0) for r, n in enumerate(sizes)]
        cat = [np.concatenate([rp[k] for rp in reps]) for k in range(1, 5)]
        for params in (dict(theta=0.5, p=4, n0=0), dict(theta=0.3, p=5, n0=0)):
            t = bhmc.Tree([dict(rp[0], **params) for rp in reps], *cat, n_per_replica=sizes)
            t.phase_ticks(reset=True)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            t.batch_sweep(seed=0, n_sweeps=1, step=1.0, use_graph=False)
            ev1.record()
            ev1.synchronize()
            # ticks of all 256 workgroups add up: per round they are the average round of one workgroup
            report("256 replicas theta=%.1f p=%d, one sweep" % (params["theta"], params["p"]),
                   t.phase_ticks(reset=True), ev0.elapsed_time(ev1) / 1000.0)
            t.close()


if __name__ == "__main__":
    main()
