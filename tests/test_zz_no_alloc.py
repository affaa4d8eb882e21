"""The allocation-free energy entry point against bhmc_energy, through the C
ABI: two calls in a row (the second on a smaller system, so the fixed scratch
array still holds the first call's larger contents), and the size limit."""
import numpy as np
import pytest

from paper_1305_1825_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1305_1825_amd import bhmc  # noqa: E402


def say(*a):
    print(*a, flush=True)


def energy_both(t, n):
    E_ref, phi_ref = t.energy(with_phi=True)
    E_dev = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda:0")
    phi = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda:0")
    t.energy_noalloc(E_dev, phi)
    torch.cuda.synchronize()
    return E_ref, phi_ref.cpu().numpy(), float(E_dev.item()), phi.cpu().numpy()


def test_energy_noalloc_matches_energy_two_calls():
    # the same kernels in the same order: the results are bit-identical
    big = W.config_colloid_10k(n=6000, p=5)
    small = W.config_colloid_10k(n=900, p=5, seed=3)
    for c in (big, small):
        n = len(c["x"])
        say("noalloc energy n=%d" % n)
        t = bhmc.Tree(c["params"], c["x"], c["y"], c["z"], c["q"])
        E_ref, phi_ref, E, phi = energy_both(t, n)
        assert E == E_ref
        assert np.array_equal(phi, phi_ref)
        # without the potential output
        E_dev = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        t.energy_noalloc(E_dev)
        torch.cuda.synchronize()
        assert float(E_dev.item()) == E_ref
        t.close()


def test_energy_noalloc_in_replica_handle_and_limit():
    sizes = [700, 1300]
    reps = [W.batched_replica(r, n) for r, n in enumerate(sizes)]
    cat = [np.concatenate([rp[k] for rp in reps]) for k in range(1, 5)]
    t = bhmc.Tree([rp[0] for rp in reps], *cat, n_per_replica=sizes)
    for r in (1, 0):
        E_ref = t.energy(replica=r)
        E_dev = torch.zeros(1, dtype=torch.float64, device="cuda:0")
        t.energy_noalloc(E_dev, replica=r)
        torch.cuda.synchronize()
        assert float(E_dev.item()) == E_ref
    with pytest.raises(bhmc.BhmcError):
        t.energy_noalloc(E_dev, replica=2)
    t.close()
    # one ion past the fixed array's capacity is rejected on the host
    n = (1 << 19) + 1
    rng = np.random.default_rng(0)
    pts = rng.random((n, 3)) * 100.0
    q = np.where(np.arange(n) % 2 == 0, 1.0, -1.0)
    P = W.make_params(box_side=100.0, p=1, leaf_cap=32)
    say("noalloc size limit")
    t = bhmc.Tree(P, pts[:, 0], pts[:, 1], pts[:, 2], q)
    with pytest.raises(bhmc.BhmcError) as e:
        t.energy_noalloc(E_dev)
    assert e.value.code == -1
    assert b"524288" in bhmc.lib().bhmc_last_error()
    t.close()
    # a null output is rejected
    lib = bhmc.lib()
    c = W.config_cube_1k(n=100)
    t = bhmc.Tree(c["params"], c["x"], c["y"], c["z"], c["q"])
    assert lib.bhmc_energy_noalloc(t.h, 0, None, None) == -1
    t.close()
