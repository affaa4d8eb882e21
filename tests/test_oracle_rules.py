"""Pins of the oracle's decision rules: the N_0 decision table of the traversal
(Sec. 3.2), the hard core of eq. 2.1 at exactly the contact distance, the hard
walls of the spherical cell and of the cube (Sec. 4), and the map from Philox
words to a trial move.

Each rule is written out here again from the paper (or from the published
Philox words) and compared with what the oracle does, on cases chosen so that
flipping one comparison (a strict for a non-strict inequality, an open for a
closed wall) changes the outcome.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1305_1825_amd import workloads as W


# ---------------------------------------------------------------- N_0 (Sec. 3.2)
def _tree_tables(t, n_src):
    cells = t.cells(moments=False)
    keys, perm = t.sorted()
    key_of = np.empty(n_src, dtype=np.uint64)
    key_of[perm] = keys
    children = {}
    for c in range(t.info()["ncell"]):
        children.setdefault(int(cells["parent"][c]), []).append(c)
    for v in children.values():
        v.sort()

    def members(c):
        lev = int(cells["level"][c])
        if lev == 0:
            return np.arange(n_src)
        sh = np.uint64(63 - 3 * lev)
        return np.nonzero((key_of >> sh) == (cells["kmin"][c] >> sh))[0]

    return cells, children, members


def _brute_decisions(cells, children, members, pts, q, x, exclude, theta, p, n0, mi, stats):
    """The paper's traversal written out: a cell with N' remaining sources is
    used through its expansion iff rho/r <= theta and N' >= N_0; otherwise it
    is opened iff N' > N_0 and it has children; otherwise every remaining
    source below it is summed directly.  Returns (phi, visited, far, near)."""
    tot = 0.0
    stats.setdefault("farabs", 0.0)
    visited = far = near = 0
    stack = [0]
    while stack:
        c = stack.pop()
        mem = [j for j in members(c) if j not in exclude]
        npr = len(mem)
        if npr == 0:
            continue
        visited += 1
        cen, h = cells["geo"][c, :3], cells["geo"][c, 3]
        d2 = float(np.sum((cen - x) ** 2))
        mac = 3 * h * h <= theta * theta * d2
        leaf = bool(cells["is_leaf"][c])
        if not mac and npr == n0 and not leaf:
            stats["at_n0_internal"] += 1
        if mac and npr == n0:
            stats["far_at_n0"] += 1
        if mac and npr >= n0:
            far += 1
            T = O.taylor(p, cen - x)
            Mp = np.zeros(len(mi))
            for j in mem:
                dd = pts[j] - cen
                Mp += q[j] * np.array([np.prod(dd ** mi[k]) for k in range(len(mi))])
            tot += float(np.dot(T, Mp))
            stats["farabs"] += float(np.sum(np.abs(T * Mp)))
        elif npr > n0 and not leaf:
            stack.extend(reversed(children[c]))
        else:
            for j in mem:
                tot += q[j] / np.linalg.norm(x - pts[j])
                near += 1
    return tot, visited, far, near


def test_n0_decision_table_by_brute_force():
    """Counts of visited, far and directly summed sources, and the potential,
    equal the decision table of Sec. 3.2 for N_0 = 1..8 (cells holding exactly
    N_0 sources occur on both sides of the MAC, so a strict / non-strict swap in
    either test changes the counts)."""
    rng = np.random.default_rng(3)
    n = 60
    pts = rng.random((n, 3)) * 10.0
    q = rng.choice([-1.0, 1.0, 2.0], size=n)
    p, theta = 3, 0.7
    mi = O.multi_indices(p)
    stats = {"at_n0_internal": 0, "far_at_n0": 0}
    for n0 in range(1, 9):
        P = W.make_params(box_side=10.0, p=p, leaf_cap=2, theta=theta, n0=n0)
        t = O.Tree(P, pts[:, 0], pts[:, 1], pts[:, 2], q)
        cells, children, members = _tree_tables(t, n)
        for tgt in range(0, n, 5):
            x = pts[tgt]
            stats["farabs"] = 0.0
            ref, vis, far, near = _brute_decisions(cells, children, members, pts, q, x, {tgt}, theta, p, n0,
                                                   mi, stats)
            phi, cnt = t.phi_counts(x, exclude=[tgt])
            assert cnt.tolist() == [vis, far, near], (n0, tgt)
            assert phi == pytest.approx(ref, rel=1e-12, abs=1e-14)
            # the far-field magnitude sum_far sum_n |T_n M'_n| the oracle reports
            assert t.far_magnitude(x, exclude=[tgt]) == pytest.approx(stats["farabs"], rel=1e-12, abs=1e-300)
    # the boundary cases the comparisons decide were exercised
    assert stats["at_n0_internal"] > 10 and stats["far_at_n0"] > 10


def test_n0_at_least_source_count_is_the_direct_sum():
    """With N_0 at least the number of remaining sources, the root is neither
    expanded nor opened: every source is summed directly (Sec. 3.2)."""
    c = W.config_colloid_10k(n=300, p=4)
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    n = len(x)
    for n0 in (2 * n - 2, 2 * n + 5):
        P = dict(c["params"], n0=n0)
        t = O.Tree(P, x, y, z, q)
        E_t, phi_t = t.energy(with_phi=True)
        phi_d = O.direct_phi(P, x, y, z, q)
        assert np.allclose(phi_t, phi_d, rtol=0, atol=1e-12 * np.abs(phi_d).max())
        for i in (0, 17, 250):
            _, cnt = t.phi_counts([x[i], y[i], z[i]], exclude=[i, n + i])
            assert cnt.tolist() == [1, 0, 2 * n - 2]


# ---------------------------------------------------------------- hard core (eq. 2.1)
def test_hard_core_at_exactly_tau_is_an_overlap():
    """V = infinity for r <= tau (eq. 2.1): a trial position at exactly tau from
    another ion is rejected as an overlap, one ulp further out it is not."""
    tau = 0.5
    P = W.make_params(box_side=20.0, hard_core=tau, leaf_cap=2, p=3)
    x = np.array([5.0, 9.0, 12.0, 3.0])
    y = np.array([5.0, 9.0, 2.0, 15.0])
    z = np.array([5.0, 9.0, 7.0, 11.0])
    q = np.array([1.0, -1.0, 1.0, -1.0])
    t = O.Tree(P, x, y, z, q)
    at = np.array([5.5, 5.0, 5.0])          # d^2 = 0.25 = tau^2 exactly
    beyond = np.array([np.nextafter(5.5, 6.0), 5.0, 5.0])
    dE, reason = t.delta(1, at)
    assert reason == 2 and math.isinf(dE)
    dE, reason = t.delta(1, beyond)
    assert reason == 0 and math.isfinite(dE)
    # the same ion never overlaps itself
    dE, reason = t.delta(0, np.array([5.25, 5.0, 5.0]))
    assert reason == 0
    # both Metropolis drivers apply the same rule: with step 0 the trial position
    # is the mover's own, and another ion sits at exactly tau from it
    i, _, _ = O.draw_move(0, 0, 0, 4, 0.0)
    j = (i + 1) % 4
    xs, ys, zs = x.copy(), y.copy(), z.copy()
    xs[j], ys[j], zs[j] = xs[i] + tau, ys[i], zs[i]
    assert (xs[j] - xs[i]) ** 2 == tau * tau
    r = O.direct_mc_run(P, xs, ys, zs, q, 0, 0, 0, 1, 0.0)
    assert r["stats"][2] == 1 and r["accept"][0] == 0
    rt = O.Tree(P, xs, ys, zs, q).mc_run(seed=0, replica=0, move0=0, n_moves=1, step=0.0)
    assert rt["stats"][2] == 1 and rt["accept"][0] == 0
    xs[j] = np.nextafter(xs[i] + tau, 20.0)
    r = O.direct_mc_run(P, xs, ys, zs, q, 0, 0, 0, 1, 0.0)
    assert r["stats"][2] == 0
    rt = O.Tree(P, xs, ys, zs, q).mc_run(seed=0, replica=0, move0=0, n_moves=1, step=0.0)
    assert rt["stats"][2] == 0


def test_tree_and_direct_chains_agree_on_hard_cores_in_the_shell():
    """Hard-core shell system: the treecode chain and the direct-sum chain
    reject the same moves for walls and overlaps (their positions are equal
    until a marginal Metropolis decision)."""
    n = 400
    q = W.colloid_charges(n, -20.0)
    x, y, z, q = W.shell_system(q, 10.5, 16.0, 0.8, seed=3)
    P = W.shell_params(10.0, -20.0, 10.5, 16.0, theta=0.4, p=8, leaf_cap=8, hard_core=0.8)
    n_moves = 600
    t = O.Tree(P, x, y, z, q)
    rt = t.mc_run(seed=5, replica=0, move0=0, n_moves=n_moves, step=1.0)
    rd = O.direct_mc_run(P, x, y, z, q, 5, 0, 0, n_moves, 1.0)
    px, py, pz = x.copy(), y.copy(), z.copy()
    overlaps = walls = 0
    tau2 = P["hard_core"] ** 2
    for k in range(n_moves):
        i, d, al = O.draw_move(5, 0, k, n, 1.0)
        rn = np.array([px[i], py[i], pz[i]]) + d
        r2 = rn[0] * rn[0] + rn[1] * rn[1] + rn[2] * rn[2]
        wall = r2 <= P["r_min"] ** 2 or r2 >= P["r_max"] ** 2
        dd = (rn[0] - px) ** 2 + (rn[1] - py) ** 2 + (rn[2] - pz) ** 2
        dd[i] = np.inf
        ovl = (not wall) and bool(np.any(dd <= tau2))
        assert math.isinf(rt["dE"][k]) == math.isinf(rd["dE"][k]) == (wall or ovl), k
        walls += wall
        overlaps += ovl
        if not (wall or ovl):
            margin = abs(math.log(al) + rd["dE"][k]) if al > 0 else 1.0
            if abs(rt["dE"][k] - rd["dE"][k]) > 0.1 * margin:
                break
            assert rt["accept"][k] == rd["accept"][k]
            if rd["accept"][k]:
                px[i], py[i], pz[i] = rn
    else:
        k = n_moves
    assert k > 300 and overlaps > 3 and walls > 0


# ---------------------------------------------------------------- walls (Sec. 4)
def test_shell_walls_reject_at_both_radii():
    """Ions are confined to r_min < |r| < r_max: a move to exactly r_min or
    exactly r_max is a wall rejection; one ulp inside is not."""
    P = W.shell_params(10.0, -5.0, 10.5, 40.0)
    x = np.array([20.0, -20.0, 0.0, 0.0])
    y = np.array([0.0, 0.0, 25.0, -25.0])
    z = np.array([0.0, 5.0, 0.0, 3.0])
    q = np.array([1.0, -1.0, 1.0, -1.0])
    t = O.Tree(P, x, y, z, q)
    for r in (10.5, 40.0):
        dE, reason = t.delta(0, np.array([r, 0.0, 0.0]))
        assert reason == 1 and math.isinf(dE)
        dE, reason = t.delta(0, np.array([0.0, 0.0, -r]))
        assert reason == 1
    for r in (np.nextafter(10.5, 11.0), np.nextafter(40.0, 39.0)):
        dE, reason = t.delta(0, np.array([r, 0.0, 0.0]))
        assert reason == 0 and math.isfinite(dE)
    with pytest.raises(O.OracleError):
        t.commit(0, np.array([40.0, 0.0, 0.0]))


def test_cube_walls_half_open():
    """The cube confinement is the root cube [lo, lo + S)^3: a move to lo is
    inside, a move to lo + S is a wall rejection."""
    P = W.make_params(box_side=20.0, p=2, leaf_cap=2)
    x = np.array([1.0, 7.0, 13.0])
    y = np.array([2.0, 8.0, 14.0])
    z = np.array([3.0, 9.0, 15.0])
    q = np.array([1.0, -1.0, 1.0])
    t = O.Tree(P, x, y, z, q)
    _, reason = t.delta(0, np.array([0.0, 2.0, 3.0]))
    assert reason == 0
    _, reason = t.delta(0, np.array([20.0, 2.0, 3.0]))
    assert reason == 1
    _, reason = t.delta(0, np.array([np.nextafter(20.0, 0.0), 2.0, 3.0]))
    assert reason == 0
    _, reason = t.delta(0, np.array([1.0, np.nextafter(0.0, -1.0), 3.0]))
    assert reason == 1


# ---------------------------------------------------------------- the trial-move map
def test_move_draw_map_from_philox_words():
    """The move of index m of replica r is the documented function of the twelve
    Philox4x32-10 words of counters (lo m, hi m, r, t), t = 0, 1, 2, recomputed
    here in exact integer arithmetic: ion (w0 N) >> 32, displacement
    step (u - 1/2) with u from (w2, w3), (w4, w5), (w6, w7), alpha from
    (w8, w9), u(a, b) = ((a >> 5) 2^26 + (b >> 6)) / 2^53."""
    def u53(a, b):
        return ((int(a) >> 5) * 2 ** 26 + (int(b) >> 6)) / 2.0 ** 53

    cases = [(0, 0, 0, 1000, 1.0), (7, 5, 123456789012, 10000, 0.5), (2 ** 64 - 1, 255, 2 ** 40 + 3, 3, 2.0),
             (0xdeadbeef12345678, 17, 999, 199999, 1.0)]
    for seed, r, m, n, step in cases:
        key = [seed & 0xFFFFFFFF, seed >> 32]
        w = np.concatenate([O.philox([m & 0xFFFFFFFF, m >> 32, r, t], key) for t in range(3)])
        i, d, al = O.draw_move(seed, r, m, n, step)
        assert i == (int(w[0]) * n) >> 32
        assert d[0] == step * (u53(w[2], w[3]) - 0.5)
        assert d[1] == step * (u53(w[4], w[5]) - 0.5)
        assert d[2] == step * (u53(w[6], w[7]) - 0.5)
        assert al == u53(w[8], w[9])
