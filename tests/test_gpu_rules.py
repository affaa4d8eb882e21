"""The decision rules on the HIP path at their boundaries, against the oracle
and the paper: the N_0 decision table of Sec. 3.2 (N_0 = 1..8), the hard core
of eq. 2.1 at exactly tau, the shell walls at exactly r_min and r_max, the
half-open cube, and a hard-core shell chain bit-exact with the oracle's."""
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


@pytest.mark.parametrize("n0", [1, 2, 3, 5, 8])
def test_delta_energy_n0_table(n0):
    """Small trees where cells of exactly N_0 sources lie on both sides of the
    MAC: the energy change equals the oracle's within the parity tolerance."""
    rng = np.random.default_rng(3)
    n = 60
    pts = rng.random((n, 3)) * 10.0
    q = rng.choice([-1.0, 1.0, 2.0], size=n)
    P = W.make_params(box_side=10.0, p=3, leaf_cap=2, theta=0.7, n0=n0)
    say("n0 table", n0)
    g = bhmc.Tree(P, pts[:, 0], pts[:, 1], pts[:, 2], q)
    o = O.Tree(P, pts[:, 0], pts[:, 1], pts[:, 2], q)
    checked = 0
    for m in range(60):
        i, d, _ = O.draw_move(17, 0, m, n, 2.0)
        rn = pts[i] + d
        dEo, ro = o.delta(i, rn)
        dEg, rg = g.delta_energy(i, rn)
        assert rg == ro
        if ro:
            continue
        scale = max(abs(dEo), abs(q[i]) * abs(o.phi(pts[i], [i])))
        assert abs(dEg - dEo) <= 1e-11 * scale, (m, dEg, dEo)
        checked += 1
    assert checked > 30
    g.close()


def test_hard_core_at_exactly_tau():
    tau = 0.5
    P = W.make_params(box_side=20.0, hard_core=tau, leaf_cap=2, p=3)
    x = np.array([5.0, 9.0, 12.0, 3.0])
    y = np.array([5.0, 9.0, 2.0, 15.0])
    z = np.array([5.0, 9.0, 7.0, 11.0])
    q = np.array([1.0, -1.0, 1.0, -1.0])
    g = bhmc.Tree(P, x, y, z, q)
    dE, reason = g.delta_energy(1, [5.5, 5.0, 5.0])     # d^2 = tau^2 exactly: V = inf (eq. 2.1)
    assert reason == bhmc.REASON_OVERLAP and math.isinf(dE)
    dE, reason = g.delta_energy(1, [np.nextafter(5.5, 6.0), 5.0, 5.0])
    assert reason == 0 and math.isfinite(dE)
    dE, reason = g.delta_energy(0, [5.25, 5.0, 5.0])    # never with itself
    assert reason == 0
    with pytest.raises(bhmc.BhmcError) as e:
        g.commit_move(1, [5.5, 5.0, 5.0])
    assert e.value.code == -3
    # a Metropolis chain with step 0 proposes the mover's own position: at exactly tau from
    # another ion it is an overlap rejection
    i, _, _ = O.draw_move(0, 0, 0, 4, 0.0)
    j = (i + 1) % 4
    xs = x.copy()
    ys, zs = y.copy(), z.copy()
    xs[j], ys[j], zs[j] = xs[i] + tau, ys[i], zs[i]
    g2 = bhmc.Tree(P, xs, ys, zs, q)
    r = g2.mc_run(seed=0, n_moves=1, step=0.0)
    assert r["rejected_overlap"] == 1
    g.close()
    g2.close()


def test_shell_walls_at_exactly_both_radii():
    P = W.shell_params(10.0, -5.0, 10.5, 40.0)
    x = np.array([20.0, -20.0, 0.0, 0.0])
    y = np.array([0.0, 0.0, 25.0, -25.0])
    z = np.array([0.0, 5.0, 0.0, 3.0])
    q = np.array([1.0, -1.0, 1.0, -1.0])
    g = bhmc.Tree(P, x, y, z, q)
    o = O.Tree(P, x, y, z, q)
    for r in (10.5, 40.0):
        for rn in ([r, 0.0, 0.0], [0.0, 0.0, -r]):
            dE, reason = g.delta_energy(0, rn)
            assert reason == bhmc.REASON_WALL and math.isinf(dE)
    for r in (np.nextafter(10.5, 11.0), np.nextafter(40.0, 39.0)):
        dE, reason = g.delta_energy(0, [r, 0.0, 0.0])
        dEo, ro = o.delta(0, [r, 0.0, 0.0])
        assert reason == ro == 0
        assert abs(dE - dEo) <= 1e-11 * max(abs(dEo), abs(o.phi([20.0, 0.0, 0.0], [0, 4])))
    with pytest.raises(bhmc.BhmcError) as e:
        g.commit_move(0, [40.0, 0.0, 0.0])
    assert e.value.code == -1
    g.close()


def test_cube_walls_half_open():
    P = W.make_params(box_side=20.0, p=2, leaf_cap=2)
    x = np.array([1.0, 7.0, 13.0])
    y = np.array([2.0, 8.0, 14.0])
    z = np.array([3.0, 9.0, 15.0])
    q = np.array([1.0, -1.0, 1.0])
    g = bhmc.Tree(P, x, y, z, q)
    assert g.delta_energy(0, [0.0, 2.0, 3.0])[1] == 0
    assert g.delta_energy(0, [20.0, 2.0, 3.0])[1] == bhmc.REASON_WALL
    assert g.delta_energy(0, [np.nextafter(20.0, 0.0), 2.0, 3.0])[1] == 0
    assert g.delta_energy(0, [1.0, np.nextafter(0.0, -1.0), 3.0])[1] == bhmc.REASON_WALL
    g.close()


def test_hard_core_shell_chain_bit_exact():
    """A dense hard-core shell system (many overlap rejections) with N_0 = 6:
    accept stream, reject reasons and positions equal the oracle's."""
    n = 400
    q = W.colloid_charges(n, -20.0)
    x, y, z, q = W.shell_system(q, 10.5, 16.0, 0.8, seed=3)
    P = W.shell_params(10.0, -20.0, 10.5, 16.0, theta=0.5, p=5, leaf_cap=8, hard_core=0.8, n0=6)
    say("hard-core shell chain")
    g = bhmc.Tree(P, x, y, z, q)
    o = O.Tree(P, x, y, z, q)
    moves = 2000
    rg = g.mc_run(seed=5, n_moves=moves, step=1.0, accept_bits=True)
    ro = o.mc_run(seed=5, replica=0, move0=0, n_moves=moves, step=1.0)
    bits = rg["accept"].cpu().numpy()
    first = np.nonzero(bits != ro["accept"])[0]
    assert len(first) == 0, "accept streams part at move %d" % first[0]
    st = ro["stats"]
    assert rg["accepted"] == st[0] and rg["rejected_wall"] == st[1] and rg["rejected_overlap"] == st[2]
    assert st[2] > 20 and st[1] > 5
    xs, ys, zs, _ = (t.cpu().numpy() for t in g.state())
    xo, yo, zo, _ = o.sources()
    assert np.array_equal(xs, xo[:n]) and np.array_equal(ys, yo[:n]) and np.array_equal(zs, zo[:n])
    g.close()
