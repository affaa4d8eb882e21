"""The multiple-image model (Kelvin image plus M line-image points per ion) on the
GPU path, through the C ABI, against the oracle.

The library computes the line rule itself (Golub-Welsch by Jacobi rotations) and
the oracle by Newton's method; both round it to multiples of 2^-40, so the image
sources, their keys and the tree must agree bit for bit.  The GPU energy keeps an
ion's own line images in its traversal and takes each back out where the
traversal met it; with N_0 = 0 that equals the oracle's exact exclusion up to
rounding, so energies and potentials are held to the tolerances of the one-image
model (1e-12 of their scale).  Moves (which move the ion, its Kelvin image and its
line images) are held to the one-image model's parity: energy changes within
1e-11, accept streams, positions and leaf index arrays bit-exact, moments within
1e-11.  The gradient (the pair terms of an ion with its own line images taken back
out as for the energy; the line images mapped back to their ion through t_m r_K and
c_m q_K) is held to the one-image gradient's parity: 1e-9 of |component| plus the
rms component."""
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


def system(n, M, theta=0.5, p=6):
    c = W.config_colloid_10k(n=n, p=p)
    return dict(c["params"], theta=theta, p=p, line_images=M), c["x"], c["y"], c["z"], c["q"]


@pytest.mark.parametrize("n,M,p", [(1500, 2, 6), (1500, 8, 6), (3000, 4, 8)])
def test_sources_tree_energy_and_potentials_match_oracle(n, M, p):
    P, x, y, z, q = system(n, M, p=p)
    say("line images n=%d M=%d p=%d" % (n, M, p))
    g = bhmc.Tree(P, x, y, z, q)
    o = O.Tree(P, x, y, z, q)
    assert g.info()["nsrc"] == (2 + M) * n
    kg, pg = g.sorted()
    ko, po = o.sorted()
    assert np.array_equal(kg, ko) and np.array_equal(pg, po)
    Eg, phig = g.energy(with_phi=True)
    Eo, phio = o.energy(with_phi=True)
    phig = phig.cpu().numpy()
    scale = 0.5 * P["l_B"] * float(np.sum(np.abs(q * phio)))
    say("  E gpu %.15g oracle %.15g" % (Eg, Eo))
    assert abs(Eg - Eo) <= 1e-12 * scale
    assert np.max(np.abs(phig - phio)) <= 1e-12 * np.max(np.abs(phio))
    # the allocation-free energy is the same computation
    Ed = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    g.energy_noalloc(Ed)
    assert abs(float(Ed.item()) - Eg) <= 1e-13 * scale
    g.close()


def test_theta_zero_is_the_direct_sum():
    P, x, y, z, q = system(800, 6, theta=0.0, p=2)
    Eg = bhmc.Tree(P, x, y, z, q).energy()
    Ed = O.direct_energy(P, x, y, z, q)
    assert abs(Eg - Ed) <= 1e-11 * abs(Ed)
    # and the line images matter: the Kelvin image alone gives another energy
    Ek = bhmc.Tree(dict(P, line_images=0), x, y, z, q).energy()
    assert abs(Ek - Ed) > 1e-3 * abs(Ed)


def test_rebuild_keeps_the_energy():
    P, x, y, z, q = system(1000, 3)
    g = bhmc.Tree(P, x, y, z, q)
    E1 = g.energy()
    g.rebuild()
    g.refresh_moments()
    assert abs(g.energy() - E1) <= 1e-13 * abs(E1)
    g.close()


def cell_map(cells):
    return {(int(l), int(k)): i for i, (l, k) in enumerate(zip(cells["level"], cells["kmin"]))}


def assert_same_slots_and_moments(g, o, p):
    """Leaf index arrays bit-exact; moments within 1e-11 of sum |q| (sqrt(3) h)^|n|."""
    cg, co = g.cells(), o.cells()
    mg, mo = cell_map(cg), cell_map(co)
    assert set(mg) == set(mo)
    members = g.leaf_members()
    lg, lo = g.leaves(), o.leaves()
    gl = {(int(cg["level"][c]), int(cg["kmin"][c])): members[l] for l, c in enumerate(lg["cell"])}
    for l in range(len(lo["cell"])):
        c = lo["cell"][l]
        key = (int(co["level"][c]), int(co["kmin"][c]))
        assert np.array_equal(gl[key], o.leaf_slots(l)), "leaf %s slots differ" % (key,)
    order = O.multi_indices(p).sum(axis=1)
    tot = np.sum(np.abs(o.sources()[3]))
    for key, io in mo.items():
        scale = tot * (np.sqrt(3.0) * co["geo"][io, 3]) ** order + 1e-300
        assert np.all(np.abs(cg["M"][mg[key]] - co["M"][io]) <= 1e-11 * scale), key


@pytest.mark.parametrize("M,p,theta", [(2, 4, 0.5), (8, 6, 0.4), (4, 8, 0.0)])
def test_energy_change_matches_oracle(M, p, theta):
    P, x, y, z, q = system(1500, M, theta=theta, p=p)
    say("line images delta M=%d p=%d theta=%g" % (M, p, theta))
    g, o = bhmc.Tree(P, x, y, z, q), O.Tree(P, x, y, z, q)
    n = len(x)
    checked = 0
    for m in range(60):
        i, d, _ = O.draw_move(321, 0, m, n, 1.5)
        rn = np.array([x[i], y[i], z[i]]) + d
        dEo, ro = o.delta(i, rn)
        dEg, rg = g.delta_energy(i, rn)
        assert rg == ro
        if ro:
            assert np.isinf(dEg)
            continue
        phi = abs(o.phi([x[i], y[i], z[i]], [i, n + i] + [2 * n + k * n + i for k in range(M)]))
        tol = 1e-11 * max(abs(dEo), P["l_B"] * abs(q[i]) * phi)
        assert abs(dEg - dEo) <= tol, (m, i, dEg, dEo)
        checked += 1
    assert checked > 40
    g.close()


@pytest.mark.parametrize("case", ["M2_p5", "M8_p6", "tight_slots"])
def test_chain_bit_exact_against_oracle(case):
    """Accept stream, statistics (rebuilds included), positions and leaf index arrays
    bit-exact; moments and the energy after the chain to their tolerances."""
    if case == "M2_p5":
        (P, x, y, z, q), moves = system(1500, 2, theta=0.4, p=5), 1500
    elif case == "M8_p6":
        (P, x, y, z, q), moves = system(1500, 8, theta=0.5, p=6), 1000
    else:  # leaves fill up: the capacity check over all 2 + M moved sources, and rebuilds
        P, x, y, z, q = system(600, 2, theta=0.5, p=5)
        P = dict(P, leaf_cap=4, slot_slack=1, max_depth=2)
        moves = 3000
    step = 2.0 if case == "tight_slots" else 1.0
    say("line images chain", case)
    g, o = bhmc.Tree(P, x, y, z, q), O.Tree(P, x, y, z, q)
    assert g.set_moves_per_round(0) == 1  # one move per traversal with line images
    rg = g.mc_run(seed=4, n_moves=moves, step=step, accept_bits=True)
    ro = o.mc_run(seed=4, replica=0, move0=0, n_moves=moves, step=step)
    first = np.nonzero(rg["accept"].cpu().numpy() != ro["accept"])[0]
    assert len(first) == 0, "accept streams part at move %d" % first[0]
    st = ro["stats"]
    assert rg["accepted"] == st[0] and rg["rejected_wall"] == st[1] and rg["rejected_overlap"] == st[2]
    assert rg["rebuilds"] == st[3]
    if case == "tight_slots":
        assert st[3] > 0
    n = len(x)
    xs, ys, zs, _ = (t.cpu().numpy() for t in g.state())
    xo, yo, zo, _ = o.sources()
    assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    assert_same_slots_and_moments(g, o, P["p"])
    Eg, Eo = g.energy(), o.energy()
    assert abs(Eg - Eo) <= 1e-11 * abs(Eo)
    g.close()


def test_chain_at_theta_zero_is_the_direct_chain():
    P, x, y, z, q = system(700, 5, theta=0.0, p=3)
    g = bhmc.Tree(P, x, y, z, q)
    rg = g.mc_run(seed=9, n_moves=1500, step=1.0, accept_bits=True)
    rd = O.direct_mc_run(P, x, y, z, q, 9, 0, 0, 1500, 1.0)
    assert np.array_equal(rg["accept"].cpu().numpy(), rd["accept"])
    xs, ys, zs, _ = (t.cpu().numpy() for t in g.state())
    assert np.array_equal(xs, rd["x"]) and np.array_equal(ys, rd["y"]) and np.array_equal(zs, rd["z"])
    g.close()


def test_commit_move_api_matches_oracle():
    P, x, y, z, q = system(800, 3, theta=0.5, p=4)
    g, o = bhmc.Tree(P, x, y, z, q), O.Tree(P, x, y, z, q)
    n = len(x)
    done = 0
    for m in range(80):
        i, d, _ = O.draw_move(77, 0, m, n, 1.0)
        xo, yo, zo, _ = o.sources()
        rn = np.array([xo[i], yo[i], zo[i]]) + d
        _, reason = o.delta(i, rn)
        if reason:
            continue
        o.commit(i, rn)
        g.commit_move(i, rn)
        done += 1
    assert done > 60
    assert_same_slots_and_moments(g, o, P["p"])
    g.close()


def test_batched_replicas_with_line_images_equal_single_chains():
    sizes = [300, 500, 420]
    reps = []
    for r, n in enumerate(sizes):
        c = W.config_colloid_10k(n=n, p=4)
        reps.append((dict(c["params"], theta=0.5, p=4, line_images=r + 1), c["x"], c["y"], c["z"], c["q"]))
    cat = [np.concatenate([rp[k] for rp in reps]) for k in range(1, 5)]
    g = bhmc.Tree([rp[0] for rp in reps], *cat, n_per_replica=sizes)
    say("  autotune", g.autotune(seed=5, step=1.0, trial_moves=100))
    stats = g.batch_sweep(seed=11, n_sweeps=2, step=1.0, use_graph=True)
    for r, (P, x, y, z, q) in enumerate(reps):
        o = O.Tree(P, x, y, z, q)
        ro = o.mc_run(seed=11, replica=r, move0=0, n_moves=2 * sizes[r], step=1.0)
        assert stats[r]["moves"] == 2 * sizes[r] and stats[r]["accepted"] == ro["stats"][0], r
        xs, ys, zs, _ = (t.cpu().numpy() for t in g.state(r))
        xo, yo, zo, _ = o.sources()
        n = sizes[r]
        assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n]), r
    g.close()


def rel_err(g, ref):
    scale = np.abs(ref) + np.sqrt(np.mean(ref ** 2)) + 1e-300
    return float(np.max(np.abs(g - ref) / scale))


@pytest.mark.parametrize("M,p,theta", [(2, 5, 0.5), (6, 4, 0.4), (8, 8, 0.5)])
def test_gradient_matches_oracle(M, p, theta):
    P, x, y, z, q = system(1200, M, theta=theta, p=p)
    say("line images gradient M=%d p=%d theta=%g" % (M, p, theta))
    g, o = bhmc.Tree(P, x, y, z, q), O.Tree(P, x, y, z, q)
    Eg, dr, dq = g.energy_grad()
    Eo, dro, dqo = o.grad()
    e_r, e_q = rel_err(dr.cpu().numpy(), dro), rel_err(dq.cpu().numpy(), dqo)
    say("  max rel err dE/dr %.3e dE/dq %.3e" % (e_r, e_q))
    assert e_r <= 1e-9 and e_q <= 1e-9
    _, phio = o.energy(with_phi=True)
    mag = P["l_B"] * 0.5 * np.sum(np.abs(q * phio))
    assert abs(Eg - g.energy()) <= 1e-13 * mag, "the gradient call's energy differs from bhmc_energy"
    assert abs(Eg - Eo) <= 1e-13 * mag + 1e-12 * abs(Eo)
    g.close()


def test_gradient_theta0_is_the_direct_gradient():
    P, x, y, z, q = system(600, 5, theta=0.0, p=3)
    g = bhmc.Tree(P, x, y, z, q)
    _, dr, dq = g.energy_grad()
    gr, gq = O.direct_grad(P, x, y, z, q)
    assert rel_err(dr.cpu().numpy(), gr) <= 1e-11
    assert rel_err(dq.cpu().numpy(), gq) <= 1e-11
    g.close()


def test_gradient_after_moves_matches_oracle():
    """The gradient on incrementally repaired moments, line images moved by the chain."""
    P, x, y, z, q = system(900, 3, theta=0.5, p=5)
    g, o = bhmc.Tree(P, x, y, z, q), O.Tree(P, x, y, z, q)
    g.mc_run(seed=2, n_moves=600, step=1.0)
    o.mc_run(seed=2, replica=0, move0=0, n_moves=600, step=1.0)
    _, dr, dq = g.energy_grad()
    _, dro, dqo = o.grad()
    assert rel_err(dr.cpu().numpy(), dro) <= 1e-9 and rel_err(dq.cpu().numpy(), dqo) <= 1e-9
    g.close()


def test_full_size_bench_configuration():
    """The bench's multiple-image workload (N = 10^4 colloid ions, M = 4, theta = 0.4,
    p = 6): energy and a 2000-move chain against the oracle; the gradient by the Euler
    identity in the charges and by central differences of the GPU energy on sampled
    components (the oracle's full gradient at this size takes minutes)."""
    c = W.config_colloid_10k()
    P = dict(c["params"], theta=0.4, p=6, n0=0, line_images=4)
    x, y, z, q = (np.array(c[k], dtype=float) for k in "xyzq")
    say("line images full size: N=%d M=4" % len(x))
    g, o = bhmc.Tree(P, x, y, z, q), O.Tree(P, x, y, z, q)
    Eg = g.energy()
    Eo, phio = o.energy(with_phi=True)
    mag = P["l_B"] * 0.5 * np.sum(np.abs(q * phio))
    assert abs(Eg - Eo) <= 1e-13 * mag + 1e-12 * abs(Eo)
    E2, dr, dq = g.energy_grad()
    assert abs(E2 - Eg) <= 1e-13 * mag
    dr, dq = dr.cpu().numpy(), dq.cpu().numpy()
    Elin = P["l_B"] * P["Q_center"] * np.sum(q / np.sqrt(x * x + y * y + z * z))
    assert abs(np.dot(q, dq) - (2 * (E2 - Elin) + Elin)) <= 1e-11 * mag
    rms = np.sqrt(np.mean(dr ** 2))
    h, bad = 1e-6, 0
    for i in W.sample_indices(len(x), 6, tag=11):
        for comp, arr in enumerate((x, y, z)):
            a1, a2 = arr.copy(), arr.copy()
            a1[i] += h
            a2[i] -= h
            args1 = [a1 if k == comp else (x, y, z)[k] for k in range(3)]
            args2 = [a2 if k == comp else (x, y, z)[k] for k in range(3)]
            fd = (bhmc.Tree(P, *args1, q).energy() - bhmc.Tree(P, *args2, q).energy()) / (2 * h)
            if abs(fd - dr[i, comp]) > 1e-6 * (abs(dr[i, comp]) + rms):
                bad += 1
    assert bad <= 1  # a shift across a MAC or cell boundary changes the interaction list
    rg = g.mc_run(seed=0, n_moves=2000, step=1.0, accept_bits=True)
    ro = o.mc_run(seed=0, replica=0, move0=0, n_moves=2000, step=1.0)
    assert np.array_equal(rg["accept"].cpu().numpy(), ro["accept"])
    xs, ys, zs, _ = (t.cpu().numpy() for t in g.state())
    xo, yo, zo, _ = o.sources()
    n = len(x)
    assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    assert abs(g.energy() - o.energy()) <= 1e-11 * mag
    g.close()
