"""Structure of the electric double layer sampled by the treecode Monte Carlo
chain: the radial distribution g(r) of the counterions around the macroion and
the integrated charge distribution Q(r) (the analogue of the paper's Fig. 6,
Sec. 4).

For ions in the spherical cell r_min < |r| < R_cell around a macroion of
charge Q_M at the centre:

    Q(r) = Q_M + sum_{i : |r_i| < r} q_i       (Q(a) = Q_M; Q(R_cell) = 0 in a neutral cell)
    g(r) = n(r) / n_0,  n(r) the counterion number density in the shell at r and
           n_0 = N / (4/3 pi (R_cell^3 - r_min^3)) the mean density of the cell.

Sampling runs the chain on the device (bhmc mc_run, one sweep = N trial moves)
and reads the positions back after every sweep; the histograms are the only
host work.  Averages come with a standard error from block averages.

    python -m paper_1305_1825_amd.observables [--n 800] [--sweeps 1000] [--p 2 6]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import workloads as W


def cell_system(n: int = 800, seed: int = 0, theta: float = 0.5, p: int = 6, valence: float = 2.0):
    """The paper's spherical cell: counterions of valence 2 and contact distance 4
    around a macroion of radius 30 and charge -2N, cell radius 80, l_B = 7.14,
    no images (Sec. 4)."""
    q = np.full(n, valence)
    x, y, z, q = W.shell_system(q, 32.0, 80.0, 4.0, seed=seed, tag=7)
    P = W.make_params(l_B=7.14, theta=theta, p=p, leaf_cap=8, geom=1, images=0, a=30.0,
                      Q_center=-valence * n, r_min=32.0, r_max=80.0, box_lo=(-80.0,) * 3, box_side=160.0,
                      hard_core=4.0)
    return P, x, y, z, q


def integrated_charge(r, q, Q_M, radii):
    """Q(r) at each radius: Q_M plus the charge of the ions with |r_i| < r."""
    order = np.argsort(r)
    rs, cq = r[order], np.cumsum(q[order])
    k = np.searchsorted(rs, radii, side="left")  # ions strictly inside
    return Q_M + np.concatenate([[0.0], cq])[k]


def radial_density(r, edges):
    """Number density of ions in the spherical shells between consecutive edges."""
    counts, _ = np.histogram(r, bins=edges)
    vol = 4.0 / 3.0 * np.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    return counts / vol


class EdlAccumulator:
    """Per-sample Q(r) and g(r), with block averages for the standard error."""

    def __init__(self, P, n, edges, radii):
        self.P, self.n = P, n
        self.edges, self.radii = np.asarray(edges, float), np.asarray(radii, float)
        self.n0 = n / (4.0 / 3.0 * np.pi * (P["r_max"] ** 3 - P["r_min"] ** 3))
        self.Q, self.g = [], []

    def add(self, x, y, z, q):
        r = np.sqrt(x * x + y * y + z * z)
        self.Q.append(integrated_charge(r, q, self.P["Q_center"], self.radii))
        self.g.append(radial_density(r, self.edges) / self.n0)

    def result(self, blocks=8):
        out = {}
        for name, arr in (("Q", np.array(self.Q)), ("g", np.array(self.g))):
            m = arr.mean(axis=0)
            nb = min(blocks, len(arr))
            bl = np.array([b.mean(axis=0) for b in np.array_split(arr, nb)])
            err = bl.std(axis=0, ddof=1) / np.sqrt(nb) if nb > 1 else np.zeros_like(m)
            out[name] = m
            out[name + "_err"] = err
        out["samples"] = len(self.Q)
        return out


def sample_tree(P, x, y, z, q, sweeps, equil, edges, radii, seed=0, step=4.0):
    """Treecode chain on the device: equil sweeps, then one sample per sweep."""
    from . import bhmc
    n = len(x)
    t = bhmc.Tree(P, x, y, z, q)
    acc = EdlAccumulator(P, n, edges, radii)
    move = 0
    for s in range(equil + sweeps):
        t.mc_run(seed=seed, n_moves=n, step=step, move0=move)
        move += n
        if s >= equil:
            xs, ys, zs, qs = (v.cpu().numpy() for v in t.state())
            acc.add(xs, ys, zs, qs)
    t.close()
    return acc.result()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=800)
    ap.add_argument("--sweeps", type=int, default=1000)
    ap.add_argument("--equil", type=int, default=200)
    ap.add_argument("--p", type=int, nargs="+", default=[2, 6])
    args = ap.parse_args()
    edges = np.linspace(32.0, 80.0, 25)
    radii = np.array([30.0, 32.0, 33.0, 34.0, 36.0, 40.0, 48.0, 60.0, 80.0])
    for p in args.p:
        P, x, y, z, q = cell_system(args.n, p=p)
        res = sample_tree(P, x, y, z, q, args.sweeps, args.equil, edges, radii)
        print(json.dumps({"p": p, "theta": P["theta"], "radii": radii.tolist(), "Q": res["Q"].tolist(),
                          "Q_err": res["Q_err"].tolist(), "g_edges": edges.tolist(), "g": res["g"].tolist(),
                          "g_err": res["g_err"].tolist(), "samples": res["samples"]}), flush=True)


if __name__ == "__main__":
    main()
