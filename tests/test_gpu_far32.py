"""The single-precision far field (far_fp32 = 1) against the FP64 oracle.

Per far cell the evaluation of eq. 3.3 in FP32 rounds the moments (2^-24 of
each), builds each T_n of eq. 3.4 from its parents in at most 3 |n| + 2
roundings, and sums the C(p+3,3) products in FP32, so its error is at most
K 2^-24 sum_n |T_n M^n| with K = C(p+3,3) + 3p + 4; the cells' values are then
added in FP64.  The oracle reports the far-field magnitude
sum_A sum_n |T_n M'^n_A| of a target, so the bound of an energy change is
K 2^-24 l_B |q_i| (magnitude at r + magnitude at r') plus the FP64 parity
tolerance.  A chain may part from the FP64 chain only at a move whose
Metropolis margin |ln alpha + dE| is within that bound."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1305_1825_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1305_1825_amd import bhmc  # noqa: E402

EPS32 = 2.0 ** -24


def k_of(p):
    return O.nterms(p) + 3 * p + 4


def say(*a):
    print(*a, flush=True)


CASES = {
    "cube1k_p4": lambda: W.config_cube_1k(),
    "colloid2k_p6": lambda: W.config_colloid_10k(n=2000),
    "colloid1500_p8": lambda: W.config_colloid_10k(n=1500, p=8),
}


@pytest.mark.parametrize("case", list(CASES))
def test_delta_energy_and_energy_far32(case):
    c = CASES[case]()
    P = c["params"]
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    n = len(x)
    imgs = P["images"]
    g = bhmc.Tree(dict(P, far_fp32=1), x, y, z, q)
    o = O.Tree(P, x, y, z, q)
    K = k_of(P["p"])
    say("far_fp32", case)
    worst = 0.0
    for m in range(60):
        i, d, _ = O.draw_move(5, 0, m, n, 1.0)
        ro_ = np.array([x[i], y[i], z[i]])
        rn = ro_ + d
        dEo, reo = o.delta(i, rn)
        dEg, reg = g.delta_energy(i, rn)
        assert reg == reo
        if reo:
            continue
        ex = [i, n + i] if imgs else [i]
        bound = K * EPS32 * P["l_B"] * abs(q[i]) * (o.far_magnitude(rn, ex) + o.far_magnitude(ro_, ex))
        scale = max(abs(dEo), P["l_B"] * abs(q[i]) * abs(o.phi(ro_, ex)))
        assert abs(dEg - dEo) <= bound + 1e-11 * scale, (m, dEg, dEo, bound)
        worst = max(worst, abs(dEg - dEo) / bound)
    say("  largest error / bound: %.3g" % worst)
    # per-ion potentials and the energy
    Eg, phig = g.energy(with_phi=True)
    Eo, phio = o.energy(with_phi=True)
    phig = phig.cpu().numpy()
    mags = np.array([o.far_magnitude([x[k], y[k], z[k]], [k, n + k] if imgs else [k]) for k in range(n)])
    assert np.all(np.abs(phig - phio) <= K * EPS32 * mags + 1e-12 * np.abs(phio).max())
    bound_E = 0.5 * P["l_B"] * K * EPS32 * np.sum(np.abs(q) * mags)
    assert abs(Eg - Eo) <= bound_E + 1e-12 * P["l_B"] * 0.5 * np.sum(np.abs(q * phio))
    g.close()


@pytest.mark.parametrize("moves_per_round", [1, 0])
def test_chain_far32(moves_per_round):
    c = W.config_colloid_10k(n=2000)
    P = c["params"]
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    n = len(x)
    g = bhmc.Tree(dict(P, far_fp32=1), x, y, z, q)
    g.set_moves_per_round(moves_per_round)
    moves = 2000
    rg = g.mc_run(seed=0, n_moves=moves, step=1.0, accept_bits=True)
    o = O.Tree(P, x, y, z, q)
    ro = o.mc_run(seed=0, replica=0, move0=0, n_moves=moves, step=1.0)
    bits = rg["accept"].cpu().numpy()
    first = np.nonzero(bits != ro["accept"])[0]
    if len(first) == 0:
        xs, ys, zs, _ = (t.cpu().numpy() for t in g.state())
        xo, yo, zo, _ = o.sources()
        assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
        return
    k = int(first[0])
    # the chains may part only where the Metropolis margin is within the FP32 bound
    o2 = O.Tree(P, x, y, z, q)
    o2.mc_run(seed=0, replica=0, move0=0, n_moves=k, step=1.0)
    xo, yo, zo, _ = o2.sources()
    i, d, al = O.draw_move(0, 0, k, n, 1.0)
    ro_ = np.array([xo[i], yo[i], zo[i]])
    ex = [i, n + i]
    bound = k_of(P["p"]) * EPS32 * P["l_B"] * abs(q[i]) * (o2.far_magnitude(ro_ + d, ex) + o2.far_magnitude(ro_, ex))
    margin = abs(math.log(al) + ro["dE"][k])
    say("  chains part at move %d: margin %.3g, FP32 bound %.3g" % (k, margin, bound))
    assert margin <= bound + 1e-9
