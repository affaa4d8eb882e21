"""Parity at the full workload sizes, in the launch shapes the benchmark times,
on samples the oracle can follow: the first trial moves of the N = 10^4 colloid
chain (the 512-thread chain kernel), the smallest and the largest of the 256
replicas after a whole autotuned, graph-replayed sweep, and the first moves of
a 199,999-ion p = 8 replica of the large batch.  Accept streams, positions and
statistics must be bit-exact.
"""
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


def same_positions(g_state, o, n):
    xs, ys, zs = (t.cpu().numpy() for t in g_state[:3])
    xo, yo, zo, _ = o.sources()
    return np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])


def test_colloid_chain_first_moves_full_size():
    c = W.config_colloid_10k()
    moves = 3000
    say("colloid N=1e4 p=6 chain,", moves, "moves")
    g = bhmc.Tree(c["params"], c["x"], c["y"], c["z"], c["q"])
    o = O.Tree(c["params"], c["x"], c["y"], c["z"], c["q"])
    rg = g.mc_run(seed=c["seed"], n_moves=moves, step=c["step"], accept_bits=True)
    ro = o.mc_run(seed=c["seed"], replica=0, move0=0, n_moves=moves, step=c["step"])
    bits = rg["accept"].cpu().numpy()
    first = np.nonzero(bits != ro["accept"])[0]
    assert len(first) == 0, "accept streams part at move %d" % first[0]
    assert rg["accepted"] == ro["stats"][0] and rg["rejected_wall"] == ro["stats"][1]
    assert rg["rejected_overlap"] == ro["stats"][2] and rg["rebuilds"] == ro["stats"][3]
    assert same_positions(g.state(), o, len(c["x"]))


def test_replica_sweep_full_size_sampled():
    R = 256
    sizes = [int(v) for v in W.replica_sizes(R, seed=0)]
    reps = [W.batched_replica(r, n, seed=0) for r, n in enumerate(sizes)]
    cat = [np.concatenate([rp[k] for rp in reps]) for k in range(1, 5)]
    g = bhmc.Tree([rp[0] for rp in reps], *cat, n_per_replica=sizes)
    say("256 replicas, autotune", g.autotune(seed=0, step=1.0, trial_moves=64))
    st = g.batch_sweep(seed=0, n_sweeps=1, step=1.0, use_graph=True)
    for r in (int(np.argmin(sizes)), int(np.argmax(sizes))):
        P, x, y, z, q = reps[r]
        say("  replica", r, "N =", sizes[r])
        o = O.Tree(P, x, y, z, q)
        ro = o.mc_run(seed=0, replica=r, move0=0, n_moves=sizes[r], step=1.0)
        assert st[r]["moves"] == sizes[r]
        assert st[r]["accepted"] == ro["stats"][0] and st[r]["rebuilds"] == ro["stats"][3], r
        assert same_positions(g.state(r), o, sizes[r]), r


def test_large_replica_first_moves_p8():
    c0, c1 = W.config_large_asym(r=0), W.config_large_asym(r=1)
    n = len(c0["x"])
    cat = [np.concatenate([c0[k], c1[k]]) for k in ("x", "y", "z", "q")]
    g = bhmc.Tree([c0["params"], c1["params"]], *cat, n_per_replica=[n, n])
    moves = 1500
    say("199,999 ions p=8, replica 1,", moves, "moves")
    rg = g.mc_run(seed=0, n_moves=moves, step=1.0, replica=1, accept_bits=True)
    o = O.Tree(c1["params"], c1["x"], c1["y"], c1["z"], c1["q"])
    ro = o.mc_run(seed=0, replica=1, move0=0, n_moves=moves, step=1.0)
    bits = rg["accept"].cpu().numpy()
    first = np.nonzero(bits != ro["accept"])[0]
    assert len(first) == 0, "accept streams part at move %d" % first[0]
    assert same_positions(g.state(1), o, n)


def test_maximum_ion_count_with_images():
    """The largest system a handle takes: 2^22 ions plus their 2^22 Kelvin
    images (2^23 sources, a 16-level tree); the first trial moves of its
    chain must match the oracle bit for bit."""
    n = 1 << 22
    q = W.colloid_charges(n, -1000.0)
    x, y, z, q = W.shell_system(q, 20.5, 400.0, 0.0, seed=0, tag=9)
    P = W.shell_params(20.0, -1000.0, 20.5, 400.0, theta=0.5, p=2, leaf_cap=16, l_B=1.0)
    say("2^22 ions + images, p=2, 300 moves")
    g = bhmc.Tree(P, x, y, z, q)
    o = O.Tree(P, x, y, z, q)
    # the GPU sorts and counts this tree over a grid of workgroups
    kg, pg = g.sorted()
    ko, po = o.sorted()
    assert np.array_equal(kg, ko) and np.array_equal(pg, po)
    for key in ("ncell", "nleaf", "depth"):
        assert g.info()[key] == o.info()[key], key
    del kg, pg, ko, po
    rg = g.mc_run(seed=0, n_moves=300, step=1.0, accept_bits=True)
    ro = o.mc_run(seed=0, replica=0, move0=0, n_moves=300, step=1.0)
    bits = rg["accept"].cpu().numpy()
    first = np.nonzero(bits != ro["accept"])[0]
    assert len(first) == 0, "accept streams part at move %d" % first[0]
    assert rg["accepted"] == ro["stats"][0] and rg["rejected_wall"] == ro["stats"][1]
    assert same_positions(g.state(), o, n)
    g.close()
