"""Pins of the oracle's multiple-image model of the dielectric sphere (the model the
paper names in Sec. 1 and Sec. 5 without formulas).

A unit charge at y outside a sphere of radius a (eps_in inside, eps_out outside)
has the reaction potential sum_n b_n a^(2n+1) / (|y|^(n+1) |x|^(n+1)) P_n(cos angle)
with b_n = n (eps_out - eps_in) / (n eps_in + (n + 1) eps_out): the textbook
solution of Laplace's equation with continuous potential and normal displacement
on the sphere.  The oracle represents it by the Kelvin image plus M points of a
line image placed by a Gauss rule of the weight t^(sigma - 1) on [0, 1]; here the
rule is pinned by its moments (and by Gauss-Legendre at sigma = 1), the image
potential by the Legendre series itself, the treecode energy with line images by
the direct sum, a Monte Carlo move (which moves the ion, its Kelvin image and its
line images) by the difference of direct energies and the direct-sum chain, and the
gradient by finite differences and the direct gradient."""
import numpy as np
import pytest
from scipy.special import eval_legendre

import oracle as O
from paper_1305_1825_amd import workloads as W

A, EIN, EOUT = 10.0, 2.0, 80.0
SIGMA = EOUT / (EIN + EOUT)


def exact_reaction(x, y, nmax=3000):
    """The Legendre series of the reaction potential at x of a unit charge at y."""
    rx, ry = np.linalg.norm(x), np.linalg.norm(y)
    c = np.clip(np.dot(x, y) / (rx * ry), -1.0, 1.0)
    n = np.arange(nmax + 1)
    b = n * (EOUT - EIN) / (n * EIN + (n + 1) * EOUT)
    return float(np.sum(b * (A / (rx * ry)) * (A * A / (rx * ry)) ** n * eval_legendre(n, c)))


def params(M, **kw):
    P = W.shell_params(A, 0.0, 10.5, 40.0, theta=0.5, p=6, leaf_cap=8, hard_core=0.0)
    return dict(P, eps_in=EIN, eps_out=EOUT, line_images=M, Q_center=0.0, **kw)


def reaction_via_direct_phi(M, x, y):
    """G_R(x; y) from the oracle's direct potential of a two-ion system."""
    xs = np.array([x[0], y[0]]), np.array([x[1], y[1]]), np.array([x[2], y[2]])
    phi = O.direct_phi(params(M), *xs, np.array([1.0, 1.0]))
    return phi[0] - 1.0 / np.linalg.norm(np.asarray(x) - np.asarray(y))


@pytest.mark.parametrize("sigma", [0.5, 0.75, SIGMA, 1.0])
def test_line_rule_integrates_moments_exactly(sigma):
    for M in range(1, 9):
        t, w = O.line_rule(sigma, M)
        assert np.all(np.diff(t) < 0) and np.all((t > 0) & (t < 1)) and np.all(w > 0)
        for k in range(2 * M):
            assert abs(np.sum(w * t ** k) - 1.0 / (k + sigma)) <= 5e-11, (sigma, M, k)  # rounding to 2^-40
        # an M-point rule is not exact one degree further (the smallest such error here is 3.5e-10)
        assert abs(np.sum(w * t ** (2 * M)) - 1.0 / (2 * M + sigma)) > 1e-10


def test_line_rule_is_gauss_legendre_at_sigma_one():
    for M in (1, 3, 8):
        x, wl = np.polynomial.legendre.leggauss(M)
        t, w = O.line_rule(1.0, M)
        assert np.allclose(np.sort(t), (1.0 + x) / 2.0, atol=2e-12, rtol=0)
        assert np.allclose(w[np.argsort(t)], wl / 2.0, atol=2e-12, rtol=0)


PAIRS = [((12.0, 0.0, 0.0), (0.0, 13.0, 0.5)),
         ((20.0, 5.0, 1.0), (-15.0, 3.0, 2.0)),
         ((14.0, -3.0, 2.0), (11.0, 4.0, -6.0))]


@pytest.mark.parametrize("pair", range(len(PAIRS)))
def test_image_potential_converges_to_the_series(pair):
    x, y = (np.array(v) for v in PAIRS[pair])
    ex = exact_reaction(x, y)
    errs = [abs(reaction_via_direct_phi(M, x, y) - ex) / abs(ex) for M in (1, 2, 4, 8)]
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] <= 1e-9, errs
    # the Kelvin image alone keeps a net image charge (its b_0 is gamma, not 0)
    kelvin = reaction_via_direct_phi(0, x, y)
    assert abs(kelvin - ex) / abs(ex) > 1e-2


def test_image_potential_near_the_sphere():
    x, y = np.array([10.6, 0.2, 0.0]), np.array([10.7, 0.0, 0.3])
    ex = exact_reaction(x, y, nmax=20000)
    assert abs(reaction_via_direct_phi(8, x, y) - ex) / abs(ex) <= 1e-5


def test_image_kernel_is_symmetric():
    for x, y in PAIRS:
        assert abs(reaction_via_direct_phi(6, x, y) - reaction_via_direct_phi(6, y, x)) <= 1e-15


def test_self_energy_matches_the_series():
    for r, tol in ((10.8, 1e-5), (13.0, 1e-8), (25.0, 1e-10)):  # down to the 2^-40 rounding of the rule
        x = np.array([r / np.sqrt(3.0)] * 3)
        ex = 0.5 * exact_reaction(x, x, nmax=20000)
        errs = []
        for M in (2, 4, 8):
            E = O.direct_energy(dict(params(M), l_B=1.0), *(np.array([v]) for v in x), np.array([1.0]))
            errs.append(abs(E - ex) / abs(ex))
        assert errs[0] > errs[1] > errs[2] or errs[2] <= 1e-13, (r, errs)
        assert errs[2] <= tol, (r, errs)


def test_image_charges_of_an_ion_sum_to_zero_and_lie_on_the_ray():
    c = W.config_colloid_10k(n=300, p=4)
    P = dict(c["params"], line_images=5)
    t = O.Tree(P, c["x"], c["y"], c["z"], c["q"])
    xs, ys, zs, qs = t.sources()
    n = len(c["x"])
    assert len(xs) == 7 * n
    tt, ww = O.line_rule(P["eps_out"] / (P["eps_in"] + P["eps_out"]), 5)
    for i in (0, 17, n - 1):
        imgs = [n + i] + [2 * n + m * n + i for m in range(5)]
        qk = qs[n + i]
        assert abs(sum(qs[s] for s in imgs)) <= 2e-11 * abs(qk)
        for m in range(5):
            s = 2 * n + m * n + i
            assert np.allclose([xs[s], ys[s], zs[s]], tt[m] * np.array([xs[n + i], ys[n + i], zs[n + i]]),
                               rtol=0, atol=1e-15)


def test_tree_energy_with_line_images_equals_direct_at_theta0_and_converges():
    c = W.config_colloid_10k(n=400, p=4)
    P = dict(c["params"], line_images=4)
    x, y, z, q = c["x"], c["y"], c["z"], c["q"]
    Ed = O.direct_energy(P, x, y, z, q)
    E0 = O.Tree(dict(P, theta=0.0), x, y, z, q).energy()
    assert abs(E0 - Ed) <= 1e-11 * abs(Ed) + 1e-12
    # at theta = 0.5 the treecode error falls with p
    errs = [abs(O.Tree(dict(P, theta=0.5, p=p), x, y, z, q).energy() - Ed) for p in (2, 6, 10)]
    assert errs[0] > errs[1] > errs[2] and errs[2] <= 1e-6 * abs(Ed)
    # the model changes the energy: the Kelvin image alone gives another value
    Ek = O.direct_energy(dict(P, line_images=0), x, y, z, q)
    assert abs(Ek - Ed) > 1e-3 * abs(Ed)


def own_sources(n, i, M):
    return [i, n + i] + [2 * n + m * n + i for m in range(M)]


@pytest.mark.parametrize("M", [1, 4, 8])
def test_move_energy_change_is_the_difference_of_energies(M):
    """The treecode energy change at theta = 0 and the direct one both equal the
    difference of the direct energies before and after the move."""
    c = W.config_colloid_10k(n=250, p=3)
    P = dict(c["params"], line_images=M)
    x, y, z, q = (np.array(c[k]) for k in "xyzq")
    t = O.Tree(dict(P, theta=0.0), x, y, z, q)
    E0 = O.direct_energy(P, x, y, z, q)
    for i, shift in ((0, 0.7), (13, -1.1), (77, 2.5)):
        rn = np.array([x[i], y[i], z[i]]) * (1.0 + 0.02 * shift) + shift
        dEt, reason = t.delta(i, rn)
        assert reason == 0
        dEd = O.direct_delta(P, x, y, z, q, i, rn)
        x2, y2, z2 = x.copy(), y.copy(), z.copy()
        x2[i], y2[i], z2[i] = rn
        dEE = O.direct_energy(P, x2, y2, z2, q) - E0
        scale = abs(E0) + 1.0
        assert abs(dEt - dEE) <= 1e-12 * scale and abs(dEd - dEE) <= 1e-12 * scale, (i, dEt, dEd, dEE)
        # the line images change the move's energy: the Kelvin image alone gives another value
        dEk = O.direct_delta(dict(P, line_images=0), x, y, z, q, i, rn)
        assert abs(dEk - dEE) > 1e-6 * scale


def test_leaves_keep_room_for_every_image_of_a_moved_ion():
    c = W.config_colloid_10k(n=400, p=3)
    for M in (0, 3, 8):
        P = dict(c["params"], line_images=M, slot_slack=1, leaf_cap=4)
        t = O.Tree(P, c["x"], c["y"], c["z"], c["q"])
        lv = t.leaves()
        count = lv["end"] - lv["begin"]
        assert np.array_equal(lv["cap"], np.maximum(count, 4) + 2 + M)


@pytest.mark.parametrize("max_depth", [3, 21])
def test_tree_chain_with_line_images_is_the_direct_chain(max_depth):
    """At theta = 0 the treecode chain (commits of the ion, its Kelvin image and its
    line images; rebuilds when a leaf fills) is the direct-sum chain move for move,
    and the tree it leaves equals a fresh build from its positions."""
    c = W.config_colloid_10k(n=500, p=4)
    P = dict(c["params"], line_images=3, leaf_cap=4, slot_slack=1, max_depth=max_depth, theta=0.0)
    x, y, z, q = (np.array(c[k]) for k in "xyzq")
    t = O.Tree(P, x, y, z, q)
    moves = 2500
    rt = t.mc_run(4, 0, 0, moves, 3.0)
    rd = O.direct_mc_run(P, x, y, z, q, 4, 0, 0, moves, 3.0)
    assert np.array_equal(rt["accept"], rd["accept"])
    fin = np.isfinite(rd["dE"])
    assert np.array_equal(fin, np.isfinite(rt["dE"]))
    assert np.max(np.abs(rt["dE"][fin] - rd["dE"][fin])) <= 1e-12
    assert np.array_equal(rt["stats"][[0, 1, 2, 4]], rd["stats"][[0, 1, 2, 4]])
    if max_depth == 3:
        assert rt["stats"][3] > 0  # the capacity check and rebuild ran
    n = len(x)
    xs, ys, zs, qs = t.sources()
    assert np.array_equal(xs[:n], rd["x"]) and np.array_equal(ys[:n], rd["y"]) and np.array_equal(zs[:n], rd["z"])
    f = O.Tree(P, rd["x"], rd["y"], rd["z"], q)
    for a, b in zip(f.sources(), (xs, ys, zs, qs)):
        assert np.array_equal(a, b)  # the moved line images sit where a build puts them
    # moments repaired move by move equal the fresh moments of the same tree
    Mi, Mf = t.cells()["M"], t.fresh_moments()
    assert np.max(np.abs(Mi - Mf)) <= 1e-10 * np.max(np.abs(Mf))
    assert abs(t.energy() - f.energy()) <= 1e-11 * abs(f.energy())
    # every source sits in exactly one leaf slot, where its tracking says
    lv = t.leaves()
    seen = np.concatenate([t.leaf_slots(l) for l in range(len(lv["cell"]))])
    assert np.array_equal(np.sort(seen), np.arange(len(xs)))


def _fd(E, arrs, i, comp, h):
    a1 = [a.copy() for a in arrs]
    a2 = [a.copy() for a in arrs]
    a1[comp][i] += h
    a2[comp][i] -= h
    return (E(*a1) - E(*a2)) / (2 * h)


@pytest.mark.parametrize("M", [2, 6])
def test_direct_gradient_with_line_images_matches_finite_differences(M):
    c = W.config_colloid_10k(n=120, p=2)
    P = dict(c["params"], line_images=M)
    arrs = [np.array(c[k], dtype=float) for k in "xyzq"]
    g, gq = O.direct_grad(P, *arrs)
    E = lambda *a: O.direct_energy(P, *a)
    for i in range(0, 120, 17):
        for comp in range(3):
            assert _fd(E, arrs, i, comp, 1e-6) == pytest.approx(g[i, comp], abs=1e-6 * (abs(g[i, comp]) + 1.0))
        assert _fd(E, arrs, i, 3, 1e-6) == pytest.approx(gq[i], abs=1e-6 * (abs(gq[i]) + 1.0))
    # the line images change the gradient: the Kelvin image alone gives another one
    gk, _ = O.direct_grad(dict(P, line_images=0), *arrs)
    assert np.max(np.abs(gk - g)) > 1e-4 * np.max(np.abs(g))


def test_tree_gradient_with_line_images():
    """theta = 0: the treecode gradient is the direct one; theta = 0.5: it matches central
    differences of the treecode energy (fresh builds), except where a shift moves a cell
    across the MAC; the Euler identity in the charges holds (E is quadratic in them plus
    the central charge's linear term)."""
    c = W.config_colloid_10k(n=200, p=4)
    P = dict(c["params"], line_images=3)
    arrs = [np.array(c[k], dtype=float) for k in "xyzq"]
    E0, g0, gq0 = O.Tree(dict(P, theta=0.0), *arrs).grad()
    gd, gqd = O.direct_grad(P, *arrs)
    assert np.allclose(g0, gd, rtol=0, atol=1e-11 * np.abs(gd).max())
    assert np.allclose(gq0, gqd, rtol=0, atol=1e-11 * np.abs(gqd).max())
    E, g, gq = O.Tree(P, *arrs).grad()
    assert E == pytest.approx(O.Tree(P, *arrs).energy(), rel=1e-14)
    x, y, z, q = arrs
    Elin = P["l_B"] * P["Q_center"] * np.sum(q / np.sqrt(x * x + y * y + z * z))
    assert np.dot(q, gq) == pytest.approx(2 * (E - Elin) + Elin, rel=1e-11)
    Et = lambda *a: O.Tree(P, *a).energy()
    rms, rmsq = np.sqrt(np.mean(g ** 2)), np.sqrt(np.mean(gq ** 2))
    bad = 0
    for i in range(0, 200, 23):
        for comp in range(3):
            if abs(_fd(Et, arrs, i, comp, 1e-6) - g[i, comp]) > 1e-6 * (abs(g[i, comp]) + rms):
                bad += 1
        assert _fd(Et, arrs, i, 3, 1e-6) == pytest.approx(gq[i], abs=1e-6 * (abs(gq[i]) + rmsq))
    assert bad <= 1


def test_oracle_line_images_parameters():
    c = W.config_colloid_10k(n=200, p=4)
    P = dict(c["params"], line_images=2)
    with pytest.raises(Exception):
        O.Tree(dict(P, line_images=9), c["x"], c["y"], c["z"], c["q"])
    with pytest.raises(Exception):
        O.Tree(dict(P, eps_in=80.0, eps_out=2.0), c["x"], c["y"], c["z"], c["q"])
