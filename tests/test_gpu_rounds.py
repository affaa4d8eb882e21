"""Chains run in rounds of several trial moves against the oracle's move-by-move
chain: accept streams, rejection reasons, positions, leaf index arrays and
moments must be those of the sequential chain (bit-exact where the oracle is,
1e-11 for moments), whatever the number of moves per round -- through rounds
cut short by a repeated ion, accepted moves that change later moves' energy
changes, overlaps with ions that moved earlier in the round, walls, and leaves
that fill up."""
import numpy as np
import pytest

import oracle as O
from paper_1305_1825_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1305_1825_amd import bhmc  # noqa: E402
from test_gpu_parity import assert_same_slots, assert_moments, cell_map  # noqa: E402


def say(*a):
    print(*a, flush=True)


def dense_shell(n=400, p=5):
    q = W.colloid_charges(n, -20.0)
    x, y, z, q = W.shell_system(q, 10.5, 16.0, 0.8, seed=3)
    P = W.shell_params(10.0, -20.0, 10.5, 16.0, theta=0.5, p=p, leaf_cap=8, hard_core=0.8)
    return P, x, y, z, q


CASES = {
    # name: (system, moves, step)
    "cube1k_p4": (lambda: (lambda c: (c["params"], c["x"], c["y"], c["z"], c["q"]))(W.config_cube_1k()), 2000, 1.0),
    "colloid2k_p6": (lambda: (lambda c: (c["params"], c["x"], c["y"], c["z"], c["q"]))(
        W.config_colloid_10k(n=2000)), 2000, 1.0),
    "colloid1500_p8": (lambda: (lambda c: (c["params"], c["x"], c["y"], c["z"], c["q"]))(
        W.config_colloid_10k(n=1500, p=8)), 1200, 1.0),
    "colloid800_p10": (lambda: (lambda c: (c["params"], c["x"], c["y"], c["z"], c["q"]))(
        W.config_colloid_10k(n=800, p=10)), 600, 1.0),
    "dense_hard_core": (lambda: dense_shell(), 3000, 1.0),
    "tight_slots": (lambda: (lambda c: (dict(c["params"], slot_slack=1, leaf_cap=4, max_depth=2), c["x"], c["y"],
                                          c["z"], c["q"]))(W.config_cube_1k()), 3000, 1.0),
    "few_ions_cube": (lambda: (W.make_params(box_side=6.0, p=3, leaf_cap=8, hard_core=0.3),
                               np.array([1.0, 2.0, 4.0, 5.0, 3.0]), np.array([1.0, 4.5, 2.0, 5.0, 3.0]),
                               np.array([1.0, 3.0, 5.0, 2.0, 3.0]), np.array([1.0, -1.0, 1.0, -1.0, 1.0])), 700, 1.5),
    "theta0_p2": (lambda: (lambda c: (dict(c["params"], theta=0.0, p=2), c["x"], c["y"], c["z"], c["q"]))(
        W.config_colloid_10k(n=600)), 800, 1.0),
}


@pytest.mark.parametrize("moves_per_round", [1, 3, 0])
@pytest.mark.parametrize("case", list(CASES))
def test_rounds_equal_sequential_oracle_chain(case, moves_per_round):
    make, moves, step = CASES[case]
    P, x, y, z, q = make()
    n = len(x)
    g = bhmc.Tree(P, x, y, z, q)
    eff = g.set_moves_per_round(moves_per_round)
    say("%s, %d moves per round" % (case, eff))
    if moves_per_round == 1:
        assert eff == 1
    o = O.Tree(P, x, y, z, q)
    rg = g.mc_run(seed=11, n_moves=moves, step=step, accept_bits=True)
    ro = o.mc_run(seed=11, replica=0, move0=0, n_moves=moves, step=step)
    bits = rg["accept"].cpu().numpy()
    first = np.nonzero(bits != ro["accept"])[0]
    assert len(first) == 0, "accept streams part at move %d" % first[0]
    st = ro["stats"]
    assert rg["accepted"] == st[0] and rg["rejected_wall"] == st[1] and rg["rejected_overlap"] == st[2]
    assert rg["rebuilds"] == st[3]
    xs, ys, zs, _ = (t.cpu().numpy() for t in g.state())
    xo, yo, zo, _ = o.sources()
    assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    assert_same_slots(g, o)
    cg, co = g.cells(), o.cells()
    assert_moments(cg, co, cell_map(cg), cell_map(co), o, P["p"], rtol=1e-11)
    if case == "tight_slots":
        assert st[3] > 0
    if case == "dense_hard_core":
        assert st[2] > 20
    g.close()


def test_rounds_in_replica_sweep():
    sizes = [1200, 2100, 1700, 900]
    reps = [W.batched_replica(r, n_r) for r, n_r in enumerate(sizes)]
    cat = [np.concatenate([rp[k] for rp in reps]) for k in range(1, 5)]
    g = bhmc.Tree([rp[0] for rp in reps], *cat, n_per_replica=sizes)
    say("4 replicas, rounds of %d moves, 3 sweeps" % g.set_moves_per_round(0))
    st = g.batch_sweep(seed=3, n_sweeps=3, step=1.0, use_graph=True)
    for k, (P, x, y, z, q) in enumerate(reps):
        o = O.Tree(P, x, y, z, q)
        ro = o.mc_run(seed=3, replica=k, move0=0, n_moves=3 * sizes[k], step=1.0)
        assert st[k]["accepted"] == ro["stats"][0] and st[k]["rebuilds"] == ro["stats"][3]
        xs, ys, zs, _ = (t.cpu().numpy() for t in g.state(k))
        xo, yo, zo, _ = o.sources()
        n = sizes[k]
        assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    g.close()


def test_rounds_need_n0_zero():
    c = W.config_colloid_10k(n=500, p=4)
    g = bhmc.Tree(dict(c["params"], n0=6), c["x"], c["y"], c["z"], c["q"])
    assert g.set_moves_per_round(0) == 1
    g.close()
    g = bhmc.Tree(c["params"], c["x"], c["y"], c["z"], c["q"])
    assert g.set_moves_per_round(0) == 8 and g.set_moves_per_round(5) == 5 and g.set_moves_per_round(1) == 1
    with pytest.raises(bhmc.BhmcError):
        g.set_moves_per_round(-1)
    g.close()
