"""Double-layer structure (the analogue of the paper's Fig. 6, Sec. 4): the
integrated charge Q(r) and the counterion distribution g(r) of the spherical
cell (N = 800 divalent counterions, macroion radius 30 and charge -1600, cell
radius 80, l_B = 7.14) sampled by the treecode chain on the GPU at theta = 0.5
with p = 2 and p = 6 agree with the same quantities sampled by the oracle's
direct-sum chain within their statistical errors; Q(a) = Q_M and
Q(R_cell) = 0 exactly.  The host helpers are pinned on hand-made
configurations."""
import numpy as np
import pytest

import oracle as O
from paper_1305_1825_amd import observables as OB


def test_integrated_charge_and_density_by_hand():
    # ions at radii 1, 2, 2, 3 with charges 1, -1, 2, 1 around Q_M = -3
    r = np.array([1.0, 2.0, 2.0, 3.0])
    q = np.array([1.0, -1.0, 2.0, 1.0])
    Q = OB.integrated_charge(r, q, -3.0, np.array([0.5, 1.0, 1.5, 2.0, 2.5, 3.5]))
    assert Q.tolist() == [-3.0, -3.0, -2.0, -2.0, -1.0, 0.0]
    edges = np.array([0.0, 1.5, 2.5, 3.5])
    dens = OB.radial_density(r, edges)
    vol = 4.0 / 3.0 * np.pi * np.array([1.5 ** 3, 2.5 ** 3 - 1.5 ** 3, 3.5 ** 3 - 2.5 ** 3])
    assert np.allclose(dens, np.array([1.0, 2.0, 1.0]) / vol, rtol=1e-15)


def direct_reference(P, x, y, z, q, sweeps, equil, edges, radii, seed, step):
    n = len(x)
    acc = OB.EdlAccumulator(P, n, edges, radii)
    xs, ys, zs = x.copy(), y.copy(), z.copy()
    for s in range(equil + sweeps):
        r = O.direct_mc_run(P, xs, ys, zs, q, seed, 0, s * n, n, step)
        xs, ys, zs = r["x"], r["y"], r["z"]
        if s >= equil:
            acc.add(xs, ys, zs, q)
    return acc.result()


@pytest.mark.gpu
@pytest.mark.parametrize("p", [2, 6])
def test_edl_structure_matches_direct_sum_chain(p):
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    n, sweeps, equil, step = 800, 600, 150, 4.0
    edges = np.linspace(32.0, 80.0, 13)
    radii = np.array([30.0, 33.0, 34.0, 36.0, 40.0, 48.0, 60.0, 80.0])
    P, x, y, z, q = OB.cell_system(n, p=p)
    print("EDL n=%d p=%d: treecode chain on the GPU" % (n, p), flush=True)
    t = OB.sample_tree(P, x, y, z, q, sweeps, equil, edges, radii, seed=1, step=step)
    print("EDL: direct-sum chain (oracle)", flush=True)
    d = direct_reference(P, x, y, z, q, sweeps, equil, edges, radii, seed=2, step=step)
    # exact: nothing inside the macroion, a neutral cell
    assert t["Q"][0] == P["Q_center"] and d["Q"][0] == P["Q_center"]
    assert abs(t["Q"][-1]) < 1e-9 and abs(d["Q"][-1]) < 1e-9
    sQ = np.sqrt(t["Q_err"] ** 2 + d["Q_err"] ** 2)
    sg = np.sqrt(t["g_err"] ** 2 + d["g_err"] ** 2)
    for k, rr in enumerate(radii):
        print("  Q(%.0f): tree %.1f +- %.1f, direct %.1f +- %.1f" % (rr, t["Q"][k], t["Q_err"][k], d["Q"][k],
                                                                   d["Q_err"][k]), flush=True)
    assert np.all(np.abs(t["Q"] - d["Q"]) <= 6.0 * sQ + 0.01 * abs(P["Q_center"]))
    assert np.all(np.abs(t["g"] - d["g"]) <= 6.0 * sg + 0.05 * np.maximum(1.0, d["g"]))
