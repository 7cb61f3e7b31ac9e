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


def test_mlp_jastrow_layout_and_width_checks():
    """The MLP Jastrow's theta entries follow jas_cusp in the generator's
    order; a width that is not a multiple of 8 or exceeds the embedding
    width is refused at handle creation."""
    import copy
    from paper_2504_06087_amd import fire
    w = wl.config(0, walkers=2)
    m = copy.deepcopy(w.model)
    m.jas_mlp_width = 16
    F = fire.Fire(w.systems[0], m, "fp64", max_walkers=2, device="cpu")
    shapes = wl.param_shapes(w.systems[0], m)
    names = [x[0] for x in F.layout]
    assert names == list(shapes.keys())
    k = names.index("jas_cusp")
    assert names[k + 1:k + 7] == ["jmlp_W1", "jmlp_b1", "jmlp_W2", "jmlp_b2", "jmlp_w3", "jmlp_b3"]
    assert all(tuple(x[2]) == tuple(shapes[x[0]]) for x in F.layout)
    for bad in (12, 64, -8):
        m.jas_mlp_width = bad
        with pytest.raises(fire.FireError):
            fire.Fire(w.systems[0], m, "fp64", max_walkers=2, device="cpu")


def test_att_jastrow_layout_and_shape_checks():
    """The attention Jastrow's theta entries follow the MLP Jastrow's in the
    generator's order; unsupported register counts, widths and readout
    widths are refused at handle creation."""
    import copy
    from paper_2504_06087_amd import fire
    w = wl.config(0, walkers=2)
    m = copy.deepcopy(w.model)
    m.jas_mlp_width = 16
    m.jas_att_regs, m.jas_att_dim, m.jas_att_width = 4, 4, 16
    F = fire.Fire(w.systems[0], m, "fp64", max_walkers=2, device="cpu")
    shapes = wl.param_shapes(w.systems[0], m)
    names = [x[0] for x in F.layout]
    assert names == list(shapes.keys())
    k = names.index("jmlp_b3")
    assert names[k + 1:k + 9] == ["jatt_q", "jatt_Wv", "jatt_W1", "jatt_b1", "jatt_W2", "jatt_b2", "jatt_w3",
                                  "jatt_b3"]
    assert all(tuple(x[2]) == tuple(shapes[x[0]]) for x in F.layout)
    for regs, dim, width in ((65, 4, 16), (4, 3, 16), (4, 4, 12), (4, 4, 264), (4, 0, 16)):
        m.jas_att_regs, m.jas_att_dim, m.jas_att_width = regs, dim, width
        with pytest.raises(fire.FireError):
            fire.Fire(w.systems[0], m, "fp64", max_walkers=2, device="cpu")


@pytest.mark.parametrize("nq,ok", [(4, True), (6, True), (12, True), (5, False), (8, False)])
def test_create_checks_the_quadrature_size(nq, ok):
    """fire_ecp_channel.n_quad names the pseudopotential rule of a species:
    4, 6 or 12 points; any other size is refused at handle creation."""
    from paper_2504_06087_amd import fire
    w = wl.config(3, walkers=2)
    s = w.systems[0]
    s.ecp_nquad = {1: nq}
    if ok:
        fire.Fire(s, w.model, "fp64", max_walkers=2, device="cpu")
    else:
        with pytest.raises(fire.FireError):
            fire.Fire(s, w.model, "fp64", max_walkers=2, device="cpu")


def test_adapt_step_is_exported_host_arithmetic():
    from paper_2504_06087_amd import fire
    out = ctypes.c_double()
    lib = fire.load()
    assert lib.fire_adapt_step(0.3, 5, 10, 0.5, 1.0, ctypes.byref(out)) == 0 and out.value == 0.3
    assert lib.fire_adapt_step(0.3, 11, 10, 0.5, 1.0, ctypes.byref(out)) != 0


def test_ecp_chunk_cap_sizes_and_errors():
    """fire_set_ecp_chunk: a negative cap or a null handle is refused; a cap
    shrinks (never grows) the workspace fire_sizes reports; 0 restores it."""
    from paper_2504_06087_amd import fire
    rng = np.random.default_rng(3)
    R, sp = wl.grown_flake(20)
    s = wl.make_system("C4H4", R, sp, pseudo_c=True, nonlocal_ecp=True, ecp_rng=rng)
    m = wl.make_model(s, width=64, mlp_layers=1, n_det=4, n_env=2, cutoff=5.0, cutoff_nuc=20.0)
    F = fire.Fire(s, m, "fp64", max_walkers=512, device="cpu")
    lib = fire.load()
    assert lib.fire_set_ecp_chunk(ctypes.c_void_p(0), 0) == -1
    assert lib.fire_set_ecp_chunk(F.h, -1) == -1
    w0 = F.sizes(512)[2]
    F.set_ecp_chunk(120)
    w1 = F.sizes(512)[2]
    F.set_ecp_chunk(0)
    assert F.sizes(512)[2] == w0
    assert w1 < w0
