"""Accuracy of the treecode against the direct sum, the measure of eq. 4.1.

For a counterion-only spherical cell shaped like the paper's Sec. 4 example
(valence 2, contact distance 4, macroion radius 30 with charge -2N, cell radius
80, l_B = 7.14, no images), prints E = sqrt(sum (V_i - V~_i)^2 / sum V_i^2) with
V_i = q_i phi_i for p = 0..10, theta in {0.5, 0.3} and several N: the
analogue of the paper's accuracy figure.  Both sides run in the HIP library:
the direct sum is the treecode at theta = 0 (every cell opened), read from
dE/dq_i = l_B phi_i + l_B Q / |r_i|.

    python -m paper_1305_1825_amd.accuracy_sweep [--n 10 100 1000 10000]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import bhmc
from . import workloads as W


def system(n: int, seed: int = 0):
    q = np.full(n, 2.0)
    x, y, z, q = W.shell_system(q, 32.0, 80.0, 4.0, seed=seed, tag=7)
    return x, y, z, q


def params(n: int, theta: float, p: int) -> dict:
    return W.make_params(l_B=7.14, theta=theta, p=p, leaf_cap=8, geom=1, images=0, a=30.0,
                         Q_center=-2.0 * n, r_min=32.0, r_max=80.0, box_lo=(-80.0,) * 3, box_side=160.0,
                         hard_core=4.0)


def direct_phi(n, x, y, z, q):
    P = params(n, 0.0, 0)
    t = bhmc.Tree(P, x, y, z, q)
    _, _, dq = t.energy_grad()
    t.close()
    r = np.sqrt(x * x + y * y + z * z)
    return (dq.cpu().numpy() - P["l_B"] * P["Q_center"] / r) / P["l_B"]


def sweep(ns, thetas=(0.5, 0.3), ps=range(11)):
    rows = []
    for n in ns:
        x, y, z, q = system(n)
        phi_d = direct_phi(n, x, y, z, q)
        V = q * phi_d
        for theta in thetas:
            for p in ps:
                t = bhmc.Tree(params(n, theta, p), x, y, z, q)
                _, phi = t.energy(with_phi=True)
                t.close()
                Vt = q * phi.cpu().numpy()
                E = float(np.sqrt(np.sum((V - Vt) ** 2) / np.sum(V ** 2)))
                rows.append({"n": n, "theta": theta, "p": p, "E": E})
                print(json.dumps(rows[-1]), flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, nargs="+", default=[10, 100, 1000, 10000])
    args = ap.parse_args()
    sweep(args.n)


if __name__ == "__main__":
    main()
