"""Direct-sum gradient of sampled ions from its closed form (test helper).

Used where the oracle's full gradient would take too long; pinned against the
oracle's direct gradient in test_direct_ref.py.
"""
import math

import numpy as np


def direct_grad_at(P, x, y, z, q, idx):
    """Closed form of the direct-sum gradient at ions idx.  By the reciprocity
    of the Kelvin image kernel, dE/dr_i = -l_B q_i F_i and dE/dq_i = l_B phi_i,
    F and phi from every ion and image but i and its own image, plus the exact
    self-image and central-charge terms."""
    l, a = P["l_B"], P["a"]
    gam = (P["eps_out"] - P["eps_in"]) / (P["eps_out"] + P["eps_in"])
    pos = np.stack([x, y, z], axis=1)
    r2 = np.sum(pos ** 2, axis=1)
    img = pos * (a * a / r2)[:, None]
    qk = gam * a * q / np.sqrt(r2)
    src = np.concatenate([pos, img]) if P["images"] else pos
    qs = np.concatenate([q, qk]) if P["images"] else q
    n = len(x)
    out_r, out_q = [], []
    for i in idx:
        keep = np.ones(len(qs), bool)
        keep[i] = False
        if P["images"]:
            keep[n + i] = False
        d = pos[i] - src[keep]
        rr = np.sqrt(np.sum(d * d, axis=1))
        phi = np.sum(qs[keep] / rr)
        F = np.sum((qs[keep] / rr ** 3)[:, None] * d, axis=0)
        gr = -l * q[i] * F
        gq = l * phi
        ri2 = r2[i]
        if P["images"]:
            den = ri2 - a * a
            gr = gr - l * gam * a * q[i] ** 2 / den ** 2 * pos[i]
            gq += l * gam * a * q[i] / den
        if P["geom"] == 1 and P["Q_center"] != 0.0:
            rn = math.sqrt(ri2)
            gr = gr - l * P["Q_center"] * q[i] / rn ** 3 * pos[i]
            gq += l * P["Q_center"] / rn
        out_r.append(gr)
        out_q.append(gq)
    return np.array(out_r), np.array(out_q)
