"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bit-exact: Morton keys, sort order, leaf ranges, leaf index arrays, Metropolis
accept streams and the positions they produce.  Floating point: the energy
change within 1e-11 of max(|dE|, l_B |q_i| |phi(r_i)|), energies and moments
within 1e-12 of their scale.
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


def both(c, **over):
    P = dict(c["params"], **over)
    g = bhmc.Tree(P, c["x"], c["y"], c["z"], c["q"])
    o = O.Tree(P, c["x"], c["y"], c["z"], c["q"])
    return P, g, o


def cell_map(cells):
    return {(int(l), int(k)): i for i, (l, k) in enumerate(zip(cells["level"], cells["kmin"]))}


def assert_same_tree(g, o):
    kg, pg = g.sorted()
    ko, po = o.sorted()
    assert np.array_equal(kg, ko), "keys differ"
    assert np.array_equal(pg, po), "sort order differs"
    cg, co = g.cells(), o.cells()
    mg, mo = cell_map(cg), cell_map(co)
    assert set(mg) == set(mo), "cell sets differ"
    for key, io in mo.items():
        assert cg["count"][mg[key]] == co["count"][io]
    lg, lo = g.leaves(), o.leaves()
    leaves_g = sorted((int(cg["level"][c]), int(cg["kmin"][c]), int(b), int(e))
                      for c, b, e in zip(lg["cell"], lg["begin"], lg["end"]))
    leaves_o = sorted((int(co["level"][c]), int(co["kmin"][c]), int(b), int(e))
                      for c, b, e in zip(lo["cell"], lo["begin"], lo["end"]))
    assert leaves_g == leaves_o, "leaf lists differ"
    return cg, co, mg, mo


def assert_same_slots(g, o):
    cg, co = g.cells(moments=False), o.cells(moments=False)
    mg = cell_map(cg)
    lg = g.leaves()
    members = g.leaf_members()
    gl = {(int(cg["level"][c]), int(cg["kmin"][c])): members[l] for l, c in enumerate(lg["cell"])}
    lo = o.leaves()
    for l in range(len(lo["cell"])):
        c = lo["cell"][l]
        key = (int(co["level"][c]), int(co["kmin"][c]))
        assert np.array_equal(gl[key], o.leaf_slots(l)), "leaf %s slots differ" % (key,)
    del mg


def assert_moments(cg, co, mg, mo, o, p, rtol=1e-12):
    mi = O.multi_indices(p)
    order = mi.sum(axis=1)
    x, y, z, q = o.sources()
    keys, perm = o.sorted()
    # scale of term n in cell A: sum_j |q_j| (sqrt(3) h)^|n|
    tot_absq = np.sum(np.abs(q))
    for key, io in mo.items():
        ig = mg[key]
        h = co["geo"][io, 3]
        scale = tot_absq * (math.sqrt(3.0) * h) ** order + 1e-300
        err = np.abs(cg["M"][ig] - co["M"][io])
        assert np.all(err <= rtol * scale), (key, np.max(err / scale))


def phi_scale(o, P, i, r):
    n = o.info()["n"]
    ex = [i, n + i] if P["images"] else [i]
    return abs(o.phi(r, ex))


# ---------------------------------------------------------------- tree build
@pytest.mark.parametrize("case", ["cube1k", "colloid2k", "colloid10k", "uniform_paper", "tiny", "colloid20k",
                                  "cube40k"])
def test_build_matches_oracle(case):
    # colloid20k (40,000 sources) and cube40k (40,000 sources, no images) are built over a
    # grid of workgroups (one replica of at least 32,768 sources), the others by one workgroup
    if case == "cube1k":
        c = W.config_cube_1k()
    elif case == "colloid20k":
        c = W.config_colloid_10k(n=20000)
    elif case == "cube40k":
        c = W.config_cube_1k(n=40000)
    elif case == "colloid2k":
        c = W.config_colloid_10k(n=2000)
    elif case == "colloid10k":
        c = W.config_colloid_10k()
    elif case == "uniform_paper":
        c = W.config_cube_1k(n=777)
        c["params"] = dict(c["params"], leaf_cap=0, max_depth=3, p=2)
    else:
        c = W.config_cube_1k(n=3)
    say("build", case)
    P, g, o = both(c)
    cg, co, mg, mo = assert_same_tree(g, o)
    assert_moments(cg, co, mg, mo, o, P["p"])
    assert_same_slots(g, o)


@pytest.mark.parametrize("n", [16384, 16385, 50001])
def test_grid_build_equals_workgroup_build(n):
    """A single large replica is sorted and counted over a grid of workgroups; a handle of
    two replicas builds both by one workgroup each.  Same keys, order, cells, leaves and slots;
    rebuilding one replica of the pair (a list of one) takes the grid path again."""
    c = W.config_colloid_10k(n=n)
    say("grid build", n)
    P = c["params"]
    g1 = bhmc.Tree(P, c["x"], c["y"], c["z"], c["q"])
    cat = [np.concatenate([c[k], c[k]]) for k in ("x", "y", "z", "q")]
    g2 = bhmc.Tree([P, P], *cat, n_per_replica=[n, n])

    def same(a, ra, b, rb):
        ka, pa = a.sorted(ra)
        kb, pb = b.sorted(rb)
        assert np.array_equal(ka, kb) and np.array_equal(pa, pb)
        ca, cb = a.cells(ra, moments=True), b.cells(rb, moments=True)
        for k in ca:
            if k == "M":
                assert np.allclose(ca[k], cb[k], rtol=1e-13, atol=1e-13 * np.max(np.abs(ca[k])))
            else:
                assert np.array_equal(ca[k], cb[k]), k
        la, lb = a.leaves(ra), b.leaves(rb)
        for k in la:
            assert np.array_equal(la[k], lb[k]), k
        # occupied slots only: a leaf's spare slots hold nothing defined
        for ma, mb in zip(a.leaf_members(ra), b.leaf_members(rb)):
            assert np.array_equal(ma, mb)

    same(g1, 0, g2, 0)
    same(g1, 0, g2, 1)
    g2.rebuild(1)
    same(g1, 0, g2, 1)
    g1.rebuild(0)
    same(g1, 0, g2, 0)
    g1.close()
    g2.close()


# ---------------------------------------------------------------- energy change and energy
@pytest.mark.parametrize("case", ["cube1k", "colloid2k_p6", "colloid_theta0", "colloid_n0", "colloid_p0",
                                  "colloid_p10", "cube_p1_theta09"])
def test_delta_energy_matches_oracle(case):
    if case == "cube1k":
        c, over = W.config_cube_1k(), {}
    elif case == "colloid2k_p6":
        c, over = W.config_colloid_10k(n=2000), {}
    elif case == "colloid_theta0":
        c, over = W.config_colloid_10k(n=500, p=3), {"theta": 0.0}
    elif case == "colloid_p0":      # lowest compiled order: monopoles only
        c, over = W.config_colloid_10k(n=800, p=0), {}
    elif case == "colloid_p10":     # highest compiled order
        c, over = W.config_colloid_10k(n=800, p=10), {}
    elif case == "cube_p1_theta09":  # the widest opening angle
        c, over = W.config_cube_1k(n=700), {"p": 1, "theta": 0.9}
    else:
        c, over = W.config_colloid_10k(n=1500, p=5), {"n0": 12}
    say("delta", case)
    P, g, o = both(c, **over)
    x, y, z = c["x"], c["y"], c["z"]
    n = len(x)
    checked = 0
    for m in range(80):
        i, d, _ = O.draw_move(123, 0, m, n, 1.0)
        rn = np.array([x[i], y[i], z[i]]) + d
        dEo, ro = o.delta(i, rn)
        dEg, rg = g.delta_energy(i, rn)
        assert rg == ro
        if ro:
            assert math.isinf(dEg)
            continue
        tol = 1e-11 * max(abs(dEo), P["l_B"] * abs(c["q"][i]) * phi_scale(o, P, i, [x[i], y[i], z[i]]))
        assert abs(dEg - dEo) <= tol, (m, i, dEg, dEo)
        checked += 1
    assert checked > 40


@pytest.mark.parametrize("case", ["cube1k", "colloid2k_p6", "colloid10k_p6"])
def test_energy_matches_oracle(case):
    c = {"cube1k": lambda: W.config_cube_1k(),
         "colloid2k_p6": lambda: W.config_colloid_10k(n=2000),
         "colloid10k_p6": lambda: W.config_colloid_10k()}[case]()
    say("energy", case)
    P, g, o = both(c)
    Eg, phig = g.energy(with_phi=True)
    Eo, phio = o.energy(with_phi=True)
    phig = phig.cpu().numpy()
    scale = np.abs(phio).max()
    assert np.all(np.abs(phig - phio) <= 1e-12 * scale)
    # E has cancellations: compare against the sum of magnitudes of its terms
    mag = P["l_B"] * 0.5 * np.sum(np.abs(c["q"] * phio))
    assert abs(Eg - Eo) <= 1e-13 * mag + 1e-12 * abs(Eo)


# ---------------------------------------------------------------- Metropolis chains
@pytest.mark.parametrize("case", ["cube1k", "colloid2k_p6", "colloid_tight_slots"])
def test_mc_chain_bit_exact(case):
    if case == "cube1k":
        c, over, moves = W.config_cube_1k(), {}, 1000
    elif case == "colloid2k_p6":
        c, over, moves = W.config_colloid_10k(n=2000), {}, 1500
    else:
        c, over, moves = W.config_cube_1k(), {"slot_slack": 1, "leaf_cap": 4, "max_depth": 2}, 3000
    say("chain", case)
    P, g, o = both(c, **over)
    rg = g.mc_run(seed=0, n_moves=moves, step=1.0, accept_bits=True)
    ro = o.mc_run(seed=0, replica=0, move0=0, n_moves=moves, step=1.0)
    bits_g = rg["accept"].cpu().numpy()
    first = np.nonzero(bits_g != ro["accept"])[0]
    assert len(first) == 0, "accept streams part at move %d" % first[0]
    st = ro["stats"]
    assert rg["accepted"] == st[0] and rg["rejected_wall"] == st[1] and rg["rejected_overlap"] == st[2]
    assert rg["rebuilds"] == st[3]
    if case == "colloid_tight_slots":
        assert st[3] > 0
    n = len(c["x"])
    xs, ys, zs, qs = (t.cpu().numpy() for t in g.state())
    xo, yo, zo, qo = o.sources()
    assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    cg, co, mg, mo = assert_same_tree(g, o) if st[3] else (None,) * 4
    assert_same_slots(g, o)
    cg, co = g.cells(), o.cells()
    assert_moments(cg, co, cell_map(cg), cell_map(co), o, P["p"], rtol=1e-11)


@pytest.mark.parametrize("case", ["cube_n4", "shell_n3_images", "cube_n40_leaf1"])
def test_mc_chain_few_ions(case):
    """Chains on a handful of ions: the same ion is drawn twice in a row on
    about every fourth move (the next mover's sources must then come from the
    committed move, not from the load made during it), chains of 700 moves
    cross several batches of drawn moves, and a one-cell tree starts its
    traversal at the root."""
    if case == "cube_n4":
        P = W.make_params(box_side=6.0, p=3, leaf_cap=8, l_B=1.0, hard_core=0.3)
        x, y, z, q = [1.0, 2.0, 4.0, 5.0], [1.0, 4.5, 2.0, 5.0], [1.0, 3.0, 5.0, 2.0], [1.0, -1.0, 1.0, -1.0]
    elif case == "shell_n3_images":
        P = W.shell_params(5.0, -3.0, 5.5, 12.0, p=4, leaf_cap=2, l_B=2.0, hard_core=0.5)
        x, y, z, q = [7.0, -6.0, 0.5], [0.5, 6.5, -8.0], [1.0, -2.0, 3.0], [1.0, 1.0, 1.0]
    else:
        c = W.config_cube_1k(n=40)
        P = dict(c["params"], leaf_cap=1, p=5)
        x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    say("few-ion chain", case)
    g = bhmc.Tree(P, x, y, z, q)
    o = O.Tree(P, x, y, z, q)
    moves = 700
    rg = g.mc_run(seed=3, n_moves=moves, step=1.5, accept_bits=True)
    ro = o.mc_run(seed=3, replica=0, move0=0, n_moves=moves, step=1.5)
    bits = rg["accept"].cpu().numpy()
    first = np.nonzero(bits != ro["accept"])[0]
    assert len(first) == 0, "accept streams part at move %d" % first[0]
    st = ro["stats"]
    assert rg["accepted"] == st[0] and rg["rejected_wall"] == st[1] and rg["rejected_overlap"] == st[2]
    assert st[0] > 50
    n = len(x)
    xs, ys, zs, _ = (t.cpu().numpy() for t in g.state())
    xo, yo, zo, _ = o.sources()
    assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    assert_same_slots(g, o)


def test_commit_move_api_and_errors():
    c = W.config_colloid_10k(n=800, p=4)
    P, g, o = both(c)
    x, y, z = c["x"].copy(), c["y"].copy(), c["z"].copy()
    n = len(x)
    done = 0
    for m in range(60):
        i, d, _ = O.draw_move(5, 0, m, n, 1.0)
        rn = np.array([x[i], y[i], z[i]]) + d
        dEo, ro = o.delta(i, rn)
        if ro == 1:
            with pytest.raises(bhmc.BhmcError) as ei:
                g.commit_move(i, rn)
            assert ei.value.code == -1
            continue
        if ro == 2:
            with pytest.raises(bhmc.BhmcError) as ei:
                g.commit_move(i, rn)
            assert ei.value.code == -3
            continue
        g.commit_move(i, rn)
        o.commit(i, rn)
        x[i], y[i], z[i] = rn
        done += 1
    assert done > 30
    assert_same_slots(g, o)
    cg, co = g.cells(), o.cells()
    assert_moments(cg, co, cell_map(cg), cell_map(co), o, P["p"], rtol=1e-11)
    with pytest.raises(bhmc.BhmcError):
        g.delta_energy(n, [11.0, 0.0, 0.0])


def test_overlap_below_far_cells():
    """Large hard core with a permissive MAC: cells within tau of the target
    can be far, and the overlap test must still see their ions."""
    c = W.config_cube_1k(n=600)
    P = dict(c["params"], theta=0.9, hard_core=1.6, leaf_cap=2)
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    # thin the system to a valid hard-core configuration
    pts = np.stack([x, y, z], axis=1)
    keep = []
    for k in range(len(pts)):
        if all(np.sum((pts[k] - pts[j]) ** 2) > 1.6 ** 2 for j in keep):
            keep.append(k)
    keep = np.array(keep)
    g = bhmc.Tree(P, x[keep], y[keep], z[keep], q[keep])
    o = O.Tree(P, x[keep], y[keep], z[keep], q[keep])
    n = len(keep)
    reasons = []
    for m in range(200):
        i, d, _ = O.draw_move(77, 0, m, n, 4.0)
        rn = np.array([x[keep][i], y[keep][i], z[keep][i]]) + d
        dEo, ro = o.delta(i, rn)
        dEg, rg = g.delta_energy(i, rn)
        assert rg == ro, (m, rg, ro)
        reasons.append(ro)
    assert reasons.count(2) > 10


def test_single_ion_and_empty_cells():
    P = W.make_params(box_side=10.0, p=3)
    g = bhmc.Tree(P, [1.0], [2.0], [3.0], [1.0])
    assert g.energy() == 0.0
    dE, r = g.delta_energy(0, [1.5, 2.0, 3.0])
    assert r == 0 and dE == 0.0
    Ps = W.shell_params(10.0, -5.0, 10.5, 20.0, p=2)
    g2 = bhmc.Tree(Ps, [12.0], [0.0], [0.0], [1.0])
    o2 = O.Tree(Ps, [12.0], [0.0], [0.0], [1.0])
    assert g2.energy() == pytest.approx(o2.energy(), rel=1e-14)
    assert g2.delta_energy(0, [13.0, 0.1, 0.0])[0] == pytest.approx(o2.delta(0, [13.0, 0.1, 0.0])[0], rel=1e-13)


def test_build_rejects_bad_input():
    P = W.make_params(box_side=10.0)
    with pytest.raises(bhmc.BhmcError) as ei:
        bhmc.Tree(P, [1.0, 11.0], [1.0, 1.0], [1.0, 1.0], [1.0, -1.0])
    assert ei.value.code == -2
    with pytest.raises(bhmc.BhmcError) as ei:
        bhmc.Tree(P, [1.0, float("nan")], [1.0, 1.0], [1.0, 1.0], [1.0, -1.0])
    assert ei.value.code == -1


# ---------------------------------------------------------------- batched replicas
@pytest.mark.parametrize("tune", [False, True])
def test_batched_replicas_equal_single_chains(tune):
    sizes = [int(v) for v in W.replica_sizes(6, seed=3, lo=200, hi=700)]
    reps = [W.batched_replica(r, n, seed=3) for r, n in enumerate(sizes)]
    Ps = [rp[0] for rp in reps]
    cat = [np.concatenate([rp[k] for rp in reps]) for k in range(1, 5)]
    say("batched", sizes, "autotuned" if tune else "")
    g = bhmc.Tree(Ps, *cat, n_per_replica=sizes)
    if tune:
        # the trials must leave every replica exactly as built
        say("  autotune", g.autotune(seed=5, step=1.0, trial_moves=100))
    stats = g.batch_sweep(seed=11, n_sweeps=2, step=1.0, use_graph=True)
    for r, (P, x, y, z, q) in enumerate(reps):
        o = O.Tree(P, x, y, z, q)
        ro = o.mc_run(seed=11, replica=r, move0=0, n_moves=2 * sizes[r], step=1.0)
        assert stats[r]["moves"] == 2 * sizes[r]
        assert stats[r]["accepted"] == ro["stats"][0], r
        xs, ys, zs, _ = (t.cpu().numpy() for t in g.state(r))
        xo, yo, zo, _ = o.sources()
        n = sizes[r]
        assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n]), r
