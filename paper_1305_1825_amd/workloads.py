"""Seeded synthetic systems for the treecode Metropolis path.

This module only draws inputs: positions, charges and parameter sets.  It holds
none of the method's arithmetic, so both the GPU library and the CPU oracle can
be fed from it.  Positions come from numpy's PCG64 stream seeded by
``(tag, replica, seed)``; the Metropolis moves themselves are drawn inside each
implementation from Philox4x32-10 keyed by the run seed.

Shapes follow the paper's numerical section (Sec. 4): ions around a fixed
spherical macroion in a spherical cell, or point charges in a cube.  Ions
carry a hard core placed by random sequential addition with resampling.
"""
from __future__ import annotations

import math

import numpy as np

try:  # scipy is only used to find hard-core conflicts quickly
    from scipy.spatial import cKDTree
except Exception:  # pragma: no cover
    cKDTree = None

BASE_PARAMS = dict(
    l_B=1.0, theta=0.5, p=4, leaf_cap=8, n0=0, max_depth=21, geom=0, images=0,
    box_lo=(0.0, 0.0, 0.0), box_side=20.0, a=0.0, Q_center=0.0, eps_in=1.0, eps_out=1.0,
    r_min=0.0, r_max=0.0, hard_core=0.0, slot_slack=2, far_fp32=0, line_images=0,
)


def make_params(**kw) -> dict:
    p = dict(BASE_PARAMS)
    for k, v in kw.items():
        if k not in p:
            raise KeyError(k)
        p[k] = v
    return p


def _rng(tag: int, replica: int, seed: int) -> np.random.Generator:
    return np.random.default_rng([int(tag), int(replica), int(seed)])


def _resolve_hard_core(pos: np.ndarray, tau: float, draw, rng, max_iter: int = 200) -> np.ndarray:
    """Redraw the later point of every pair closer than tau until none is."""
    if tau <= 0.0:
        return pos
    if cKDTree is None:
        raise RuntimeError("scipy is needed for hard-core placement")
    for _ in range(max_iter):
        pairs = cKDTree(pos).query_pairs(tau * (1.0 + 1e-9), output_type="ndarray")
        if len(pairs) == 0:
            return pos
        bad = np.unique(pairs.max(axis=1))
        pos[bad] = draw(rng, len(bad))
    raise RuntimeError("hard-core placement did not converge")


def _shell_points(rng, n, r_min, r_max):
    """Uniform in volume in r_min < r < r_max."""
    u = rng.random(n)
    r = np.cbrt(r_min ** 3 + u * (r_max ** 3 - r_min ** 3))
    v = rng.normal(size=(n, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    pts = v * r[:, None]
    # keep strictly inside the open shell after rounding
    rr = np.einsum("ij,ij->i", pts, pts)
    bad = (rr <= r_min * r_min) | (rr >= r_max * r_max)
    if bad.any():
        pts[bad] = _shell_points(rng, int(bad.sum()), r_min, r_max)
    return pts


def cube_system(n_plus: int, n_minus: int, side: float, seed: int = 0, tag: int = 1,
                replica: int = 0, hard_core: float = 0.0):
    rng = _rng(tag, replica, seed)
    n = n_plus + n_minus

    def draw(g, k):
        return g.random((k, 3)) * side

    pos = _resolve_hard_core(draw(rng, n), hard_core, draw, rng)
    q = np.concatenate([np.ones(n_plus), -np.ones(n_minus)])
    return pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), q


def shell_system(charges: np.ndarray, r_min: float, r_max: float, hard_core: float, seed: int = 0,
                 tag: int = 2, replica: int = 0):
    rng = _rng(tag, replica, seed)
    n = len(charges)

    def draw(g, k):
        return _shell_points(g, k, r_min, r_max)

    pos = _resolve_hard_core(draw(rng, n), hard_core, draw, rng)
    return pos[:, 0].copy(), pos[:, 1].copy(), pos[:, 2].copy(), np.asarray(charges, dtype=np.float64)


def shell_params(a, Q_center, r_min, r_max, **kw):
    base = dict(geom=1, images=1, a=a, Q_center=Q_center, eps_in=2.0, eps_out=80.0,
                r_min=r_min, r_max=r_max, box_lo=(-r_max, -r_max, -r_max), box_side=2.0 * r_max)
    base.update(kw)
    return make_params(**base)


# ---------------------------------------------------------------- configurations
def config_cube_1k(seed: int = 0, n: int = 1000):
    """Point charges +-1 (half each) uniform in a cube of side 20; l_B = 1,
    theta = 0.5, p = 4, leaf 8; moves uniform in [-0.5, 0.5]^3."""
    x, y, z, q = cube_system(n // 2, n - n // 2, 20.0, seed=seed)
    P = make_params(theta=0.5, p=4, leaf_cap=8, box_side=20.0)
    return dict(name="cube_N%d_p4" % n, params=P, x=x, y=y, z=z, q=q, step=1.0, moves=1000,
                seed=seed)


def colloid_charges(n: int, Q_center: float, z_plus: int = 1, z_minus: int = 1):
    """Counterions neutralising Q_center plus a symmetric z:z salt, or, for
    z_plus != z_minus, the neutral mix of the two species."""
    if z_plus == z_minus:
        excess = int(round(-Q_center / z_plus))
        n_plus = (n + excess) // 2
        n_minus = n - n_plus
    else:
        # z_plus n_plus - z_minus n_minus = -Q_center, n_plus + n_minus = n
        n_plus = int(round((z_minus * n - Q_center) / (z_plus + z_minus)))
        n_minus = n - n_plus
    q = np.concatenate([np.full(n_plus, float(z_plus)), np.full(n_minus, -float(z_minus))])
    return q


def config_colloid_10k(seed: int = 0, n: int = 10000, theta: float = 0.5, p: int = 6):
    """Sphere a = 10, Q_M = -50, eps_in/eps_out = 2/80; monovalent ions
    (50 excess counterions, rest 1:1) in 10.5 < r < 40 with hard core 0.5;
    one Kelvin image per ion; theta = 0.5, p = 6, leaf 16."""
    q = colloid_charges(n, -50.0)
    x, y, z, q = shell_system(q, 10.5, 40.0, 0.5, seed=seed)
    P = shell_params(10.0, -50.0, 10.5, 40.0, theta=theta, p=p, leaf_cap=16, hard_core=0.5)
    return dict(name="colloid_N%d_p%d" % (n, p), params=P, x=x, y=y, z=z, q=q, step=1.0,
                moves=100000, seed=seed)


def replica_sizes(R: int = 256, seed: int = 0, lo: int = 2000, hi: int = 20000):
    rng = _rng(4, 0, seed)
    n = lo + np.floor(rng.random(R) * (hi - lo + 1)).astype(np.int64)
    return (n // 2) * 2


def batched_replica(r: int, n: int, seed: int = 0):
    """One replica of the batched workload: the cube workload's species and
    parameters (+-1, theta 0.5, p 4, leaf 8) in the a = 10 sphere (eps 2/80,
    Q_M = 0), shell 10.5 < r < R_r with R_r chosen to keep the cube's number
    density 1000 / 20^3 = 0.125.  Leaf index arrays get three times their
    build-time fill: over many sweeps +-1 pairs cluster, and a full leaf stops
    the replica for a rebuild."""
    R_out = (6.0 * n / math.pi + 10.5 ** 3) ** (1.0 / 3.0)
    q = np.concatenate([np.ones(n // 2), -np.ones(n - n // 2)])
    x, y, z, q = shell_system(q, 10.5, R_out, 0.0, seed=seed, tag=4, replica=r)
    P = shell_params(10.0, 0.0, 10.5, R_out, theta=0.5, p=4, leaf_cap=8, slot_slack=3)
    return P, x, y, z, q


def config_gradient_100k(seed: int = 0, n: int = 100000, theta: float = 0.5):
    q = colloid_charges(n, -50.0)
    x, y, z, q = shell_system(q, 10.5, 120.0, 0.5, seed=seed, tag=5)
    P = shell_params(10.0, -50.0, 10.5, 120.0, theta=theta, p=6, leaf_cap=16, hard_core=0.5)
    return dict(name="grad_N%d_theta%.1f" % (n, theta), params=P, x=x, y=y, z=z, q=q)


def config_large_asym(r: int = 0, seed: int = 0, n: int = 199999):
    q = colloid_charges(n, -200.0, z_plus=2, z_minus=1)
    x, y, z, q = shell_system(q, 20.5, 200.0, 0.5, seed=seed, tag=6, replica=r)
    P = shell_params(20.0, -200.0, 20.5, 200.0, theta=0.5, p=8, leaf_cap=32, hard_core=0.5, slot_slack=3)
    return dict(name="asym_N%d_p8" % n, params=P, x=x, y=y, z=z, q=q, step=1.0)


def sample_indices(n: int, k: int, tag: int = 5, seed: int = 0) -> np.ndarray:
    """k distinct ion indices drawn uniformly (for checks on sampled outputs)."""
    return np.sort(_rng(tag, 0, seed).choice(n, size=min(k, n), replace=False))
