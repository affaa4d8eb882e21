"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/bhmc.h declares, and rejects bad parameters before it
touches any device memory."""
import ctypes as C
import os
import re

import pytest

from paper_1305_1825_amd import bhmc, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "bhmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(bhmc_[a-z_]+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_functions() == bhmc.EXPORTED


def test_library_exports_every_declared_symbol():
    L = bhmc.lib()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing


@pytest.mark.parametrize("bad", [dict(theta=1.0), dict(theta=-0.1), dict(p=11), dict(p=-1),
                                 dict(max_depth=22), dict(slot_slack=0), dict(box_side=0.0),
                                 dict(images=1), dict(geom=2), dict(leaf_cap=-1), dict(slot_slack=1025),
                                 dict(leaf_cap=(1 << 23) + 1),
                                 # shell configurations whose root cube misses part of the shell
                                 W.shell_params(10.0, 0.0, 10.5, 40.0, box_side=79.0),
                                 W.shell_params(10.0, 0.0, 10.5, 40.0, box_lo=(-40.0, -39.0, -40.0)),
                                 # the multiple-image model: M in 0..8, images on, N_0 = 0, eps_in <= eps_out
                                 dict(W.shell_params(10.0, 0.0, 10.5, 40.0), line_images=9),
                                 dict(W.shell_params(10.0, 0.0, 10.5, 40.0), line_images=-1),
                                 dict(W.shell_params(10.0, 0.0, 10.5, 40.0), line_images=2, images=0),
                                 dict(W.shell_params(10.0, 0.0, 10.5, 40.0), line_images=2, n0=4),
                                 dict(W.shell_params(10.0, 0.0, 10.5, 40.0), line_images=2, eps_in=80.0, eps_out=2.0)])
def test_parameter_validation_on_host(bad):
    P = W.make_params(**bad)
    pp = bhmc.make_params(P)
    h = C.c_void_p()
    fake = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    st = bhmc.lib().bhmc_build(C.byref(pp), 10, fake, fake, fake, fake, None, C.byref(h))
    assert st == -1
    assert h.value is None
    assert b"" != bhmc.lib().bhmc_last_error()


def test_null_inputs_rejected():
    pp = bhmc.make_params(W.make_params())
    h = C.c_void_p()
    assert bhmc.lib().bhmc_build(C.byref(pp), 10, None, None, None, None, None, C.byref(h)) == -1
    assert bhmc.lib().bhmc_build(C.byref(pp), 0, C.c_void_p(1), C.c_void_p(1), C.c_void_p(1),
                                 C.c_void_p(1), None, C.byref(h)) == -1
    # one past the largest ion count a handle takes
    assert bhmc.lib().bhmc_build(C.byref(pp), (1 << 22) + 1, C.c_void_p(1), C.c_void_p(1), C.c_void_p(1),
                                 C.c_void_p(1), None, C.byref(h)) == -1
    assert b"2^22" in bhmc.lib().bhmc_last_error()
