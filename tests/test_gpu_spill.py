"""Traversal frontiers that outgrow their on-chip capacity (Sec. 3.2's MAC
traversal, breadth first).

With the LDS capacity forced down to 64 entries every traversal streams its
wider levels through HBM regions: the energy change, the chains, the energy
and the gradient must equal the oracle's exactly as on the normal path.  With
spilling switched off the same calls return BHMC_ESTACK and leave the handle
usable.  theta = 0 (every cell opened: the direct sum) at the 10^5-ion size
needs far more frontier than the chip holds: its energy changes must equal the
direct sum's.
"""
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


def say(*a):
    print(*a, flush=True)


def rel_err(g, ref):
    scale = np.abs(ref) + np.sqrt(np.mean(ref ** 2)) + 1e-300
    return float(np.max(np.abs(g - ref) / scale))


def test_spilled_frontier_equals_oracle():
    c = W.config_colloid_10k(n=1500, p=4)
    P = dict(c["params"], theta=0.3)
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    n = len(x)
    say("forced 64-entry LDS frontier, colloid n=1500 theta=0.3")
    g = bhmc.Tree(P, x, y, z, q)
    g.set_frontier_capacity(64, allow_spill=True)
    o = O.Tree(P, x, y, z, q)
    # energy change
    for m in range(30):
        i, d, _ = O.draw_move(4, 0, m, n, 1.0)
        rn = np.array([x[i], y[i], z[i]]) + d
        dEo, ro = o.delta(i, rn)
        dEg, rg = g.delta_energy(i, rn)
        assert rg == ro
        if not ro:
            scale = max(abs(dEo), P["l_B"] * abs(q[i]) * abs(o.phi([x[i], y[i], z[i]], [i, n + i])))
            assert abs(dEg - dEo) <= 1e-11 * scale
    # energy and potentials
    Eg, phig = g.energy(with_phi=True)
    Eo, phio = o.energy(with_phi=True)
    assert np.all(np.abs(phig.cpu().numpy() - phio) <= 1e-12 * np.abs(phio).max())
    # gradient
    _, dr, dq = g.energy_grad()
    _, dro, dqo = o.grad()
    assert rel_err(dr.cpu().numpy(), dro) <= 1e-9 and rel_err(dq.cpu().numpy(), dqo) <= 1e-9
    # a chain
    rg = g.mc_run(seed=2, n_moves=600, step=1.0, accept_bits=True)
    ro = o.mc_run(seed=2, replica=0, move0=0, n_moves=600, step=1.0)
    assert np.array_equal(rg["accept"].cpu().numpy(), ro["accept"])
    xs, ys, zs, _ = (t.cpu().numpy() for t in g.state())
    xo, yo, zo, _ = o.sources()
    assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    g.close()


def test_spilled_frontier_in_replica_sweep():
    sizes = [900, 1400, 1100]
    reps = [W.batched_replica(r, n_r) for r, n_r in enumerate(sizes)]
    Ps = [dict(rp[0], theta=0.25) for rp in reps]
    cat = [np.concatenate([rp[k] for rp in reps]) for k in range(1, 5)]
    say("forced 64-entry LDS frontier, 3 replicas, 2 sweeps")
    g = bhmc.Tree(Ps, *cat, n_per_replica=sizes)
    g.set_frontier_capacity(64, allow_spill=True)
    st = g.batch_sweep(seed=1, n_sweeps=2, step=1.0, use_graph=False)
    for k, (P0, x, y, z, q) in enumerate(reps):
        o = O.Tree(Ps[k], x, y, z, q)
        ro = o.mc_run(seed=1, replica=k, move0=0, n_moves=2 * sizes[k], step=1.0)
        assert st[k]["accepted"] == ro["stats"][0]
        xs, ys, zs, _ = (t.cpu().numpy() for t in g.state(k))
        xo, yo, zo, _ = o.sources()
        n = sizes[k]
        assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    g.close()


def test_frontier_overflow_without_spill_returns_estack():
    c = W.config_colloid_10k(n=1500, p=4)
    P = dict(c["params"], theta=0.0)
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    g = bhmc.Tree(P, x, y, z, q)
    g.set_frontier_capacity(64, allow_spill=False)
    with pytest.raises(bhmc.BhmcError) as e:
        g.delta_energy(0, [x[0] + 0.1, y[0], z[0]])
    assert e.value.code == -7
    with pytest.raises(bhmc.BhmcError) as e:
        g.energy()
    assert e.value.code == -7
    with pytest.raises(bhmc.BhmcError) as e:
        g.energy_grad()
    assert e.value.code == -7
    with pytest.raises(bhmc.BhmcError) as e:
        g.mc_run(seed=0, n_moves=10, step=1.0)
    assert e.value.code == -7
    with pytest.raises(bhmc.BhmcError):
        g.set_frontier_capacity(32)
    # the handle still works once the frontier may spill again
    g.set_frontier_capacity(4096, allow_spill=True)
    o = O.Tree(P, x, y, z, q)
    assert abs(g.energy() - o.energy()) <= 1e-12 * P["l_B"] * 0.5 * np.sum(np.abs(q * o.energy(with_phi=True)[1]))
    g.close()


def test_theta_zero_direct_sum_at_1e5_ions():
    """theta = 0 opens every cell, so the treecode is the direct sum; at 10^5
    ions and their images a level holds up to ~2e4 cells, several times the
    on-chip frontier."""
    c = W.config_gradient_100k(theta=0.0)
    P = c["params"]
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    n = len(x)
    say("theta=0 at N=1e5: delta_energy against the direct sum")
    g = bhmc.Tree(P, x, y, z, q)
    checked = 0
    for m in range(25):
        i, d, _ = O.draw_move(9, 0, m, n, 1.0)
        rn = np.array([x[i], y[i], z[i]]) + d
        dEg, rg = g.delta_energy(i, rn)
        r2 = rn @ rn
        wall = r2 <= P["r_min"] ** 2 or r2 >= P["r_max"] ** 2
        if wall:
            assert rg == bhmc.REASON_WALL
            continue
        if rg:
            continue
        dEd = O.direct_delta(P, x, y, z, q, i, rn)
        # both are the exact energy change summed in different orders
        pos = np.stack([x, y, z], axis=1)
        mag = P["l_B"] * abs(q[i]) * np.sum(1.0 / np.linalg.norm(pos - np.array([x[i], y[i], z[i]]) + 1e-300,
                                                                  axis=1)[np.arange(n) != i])
        assert abs(dEg - dEd) <= 1e-11 * mag, (m, dEg, dEd)
        checked += 1
    assert checked > 15
    say("theta=0 at N=1e5: energy")
    E0 = g.energy()
    assert math.isfinite(E0)
    g.close()
