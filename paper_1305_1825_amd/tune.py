"""Opening angle and expansion order at a fixed accuracy, picked by measurement.

For one system, every (theta, p) candidate is scored by the error E of eq. 4.1
against the direct sum (the library at theta = 0) and, if E meets the target,
by the Metropolis rate of a short chain on the GPU; the fastest candidate that
meets the target wins.  The paper leaves theta, p and N_0 to the user (Sec. 4
discusses their trade-off); this makes the choice for a given system and
error.

    python -m paper_1305_1825_amd.tune [--target 1e-4] [--moves 5000]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import bhmc
from . import workloads as W


def direct_phi(P, x, y, z, q):
    t = bhmc.Tree(dict(P, theta=0.0), x, y, z, q)
    _, _, dq = t.energy_grad()
    t.close()
    dq = dq.cpu().numpy()
    l = P["l_B"]
    extra = np.zeros_like(q)
    if P.get("geom", 0) == 1:
        r2 = x * x + y * y + z * z
        if P.get("images", 0):
            gam = (P["eps_out"] - P["eps_in"]) / (P["eps_out"] + P["eps_in"])
            extra += l * gam * P["a"] * q / (r2 - P["a"] ** 2)
        extra += l * P.get("Q_center", 0.0) / np.sqrt(r2)
    return (dq - extra) / l


def error_41(P, x, y, z, q, phi_d):
    t = bhmc.Tree(P, x, y, z, q)
    _, phi = t.energy(with_phi=True)
    t.close()
    V, Vt = q * phi_d, q * phi.cpu().numpy()
    return float(np.sqrt(np.sum((V - Vt) ** 2) / np.sum(V ** 2)))


def chain_rate(P, x, y, z, q, moves, step, seed=0):
    import torch
    t = bhmc.Tree(P, x, y, z, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t.mc_run(seed=seed, n_moves=moves, step=step)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t.close()
    return moves / dt


def tune(P, x, y, z, q, target=1e-4, thetas=(0.3, 0.4, 0.5, 0.6, 0.7), ps=range(2, 11), moves=5000,
         step=1.0):
    phi_d = direct_phi(P, x, y, z, q)
    rows = []
    for theta in thetas:
        for p in ps:
            Pc = dict(P, theta=theta, p=p)
            E = error_41(Pc, x, y, z, q, phi_d)
            row = {"theta": theta, "p": p, "E": E}
            if E <= target:
                row["moves_per_s"] = chain_rate(Pc, x, y, z, q, moves, step)
            rows.append(row)
            print(json.dumps(row), flush=True)
            if E <= target:
                break  # a larger p at this theta is only slower
    ok = [r for r in rows if "moves_per_s" in r]
    best = max(ok, key=lambda r: r["moves_per_s"]) if ok else None
    return best, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--target", type=float, default=1e-4)
    ap.add_argument("--moves", type=int, default=5000)
    args = ap.parse_args()
    c = W.config_colloid_10k()
    best, _ = tune(c["params"], c["x"], c["y"], c["z"], c["q"], target=args.target, moves=args.moves,
                   step=c["step"])
    print(json.dumps({"best": best}), flush=True)


if __name__ == "__main__":
    main()
