"""The accuracy sweep (the analogue of the paper's accuracy figure, Sec. 4,
eq. 4.1) on the GPU path: the paper's p = 2 claims hold (E < 1e-2 at
theta = 0.5, E < 1e-3 at theta = 0.3) on the paper-shaped counterion cell at
N = 100 and 800, and the E the sweep reports equals the oracle's E of the same
systems (treecode and direct sum both from the oracle) within 1e-9 relative
(plus the 1e-13 to which the two direct sums agree), for p = 0, 2, 6."""
import json
import os

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1305_1825_amd import accuracy_sweep as A  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.parametrize("n", [100, 800])
def test_sweep_meets_paper_claims_and_equals_oracle(n):
    gold = json.load(open(os.path.join(HERE, "golden", "paper_accuracy_claims.json")))
    bound = {c["theta"]: c["E_below"] for c in gold["claims"]}
    rows = A.sweep([n], thetas=(0.5, 0.3), ps=(0, 2, 6))
    x, y, z, q = A.system(n)
    P0 = A.params(n, 0.0, 0)
    V = q * O.direct_phi(P0, x, y, z, q)
    for r in rows:
        if r["p"] == 2:
            assert r["E"] < bound[r["theta"]], r
        _, phi = O.Tree(A.params(n, r["theta"], r["p"]), x, y, z, q).energy(with_phi=True)
        E_o = float(np.sqrt(np.sum((V - q * phi) ** 2) / np.sum(V ** 2)))
        # both are differences of sums of size |V|, rounded at about 1e-16 of |V|
        assert abs(r["E"] - E_o) <= 1e-9 * E_o + 1e-13, (r, E_o)
