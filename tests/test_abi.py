"""The C-ABI library loads, exports every declared symbol and validates its
arguments on the host (no device compute)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "fire.h")).read()
    return sorted(set(re.findall(r"^(?:fire_status|const char\*)\s+(fire_\w+)\(", txt, re.M)))


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ["fire_eval_logpsi", "fire_mcmc_sweep", "fire_local_energy", "fire_ecp_nonlocal",
              "fire_grad_params", "fire_create", "fire_sizes", "fire_set_params"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2504_06087_amd import fire
    lib = fire.load()
    for n in _declared():
        assert hasattr(lib, n), n
    assert set(_declared()) == set(fire.EXPORTS)


@pytest.mark.parametrize("cid", [0, 1, 3])
def test_theta_layout_matches_generator(cid):
    from paper_2504_06087_amd import fire
    w = wl.config(cid, walkers=2)
    F = fire.Fire(w.systems[0], w.model, w.precision, max_walkers=8, device="cpu")
    shapes = wl.param_shapes(w.systems[0], w.model)
    assert [x[0] for x in F.layout] == list(shapes.keys())
    assert all(tuple(x[2]) == tuple(shapes[x[0]]) for x in F.layout)
    assert F.P == sum(int(np.prod(s)) for s in shapes.values())
    th = F.flatten(w.params[0])
    back = F.unflatten(th)
    for k, v in w.params[0].items():
        assert np.array_equal(back[k], v)


def test_host_side_errors():
    from paper_2504_06087_amd import fire
    w = wl.config(0, walkers=2)
    F = fire.Fire(w.systems[0], w.model, "fp64", max_walkers=8, device="cpu")
    lib = fire.load()
    p, s, ws = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.fire_sizes(F.h, 9, ctypes.byref(p), ctypes.byref(s), ctypes.byref(ws)) == -4   # W > max
    assert lib.fire_sizes(F.h, 0, ctypes.byref(p), ctypes.byref(s), ctypes.byref(ws)) == -1
    # calls before parameters are set, and null pointers, return without launching
    null = ctypes.c_void_p(0)
    dummy = ctypes.c_void_p(16)
    assert lib.fire_eval_logpsi(F.h, 2, null, dummy, dummy, null, null, dummy, null) == -1
    assert lib.fire_eval_logpsi(F.h, 2, dummy, dummy, dummy, null, null, dummy, null) == -6
    assert lib.fire_eval_logpsi(F.h, 9, dummy, dummy, dummy, null, null, dummy, null) == -4
    assert fire.fire_status_string(-4).startswith("walker count")


def test_create_rejects_unsupported_shapes():
    from paper_2504_06087_amd import fire
    w = wl.config(0, walkers=2)
    m = w.model
    m.width = 300
    with pytest.raises(fire.FireError):
        fire.Fire(w.systems[0], m, "fp64", max_walkers=8, device="cpu")
