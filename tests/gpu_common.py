"""Helpers of the GPU parity tests: build a handle and the oracle on the same
seeded workload."""
import copy
import sys

import numpy as np
import torch

import workloads as wl


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def setup(cid, W, precision=None, model_kw=None, system_fn=None, **fire_kw):
    from oracle import Oracle
    from paper_2504_06087_amd import fire
    w = wl.config(cid, walkers=W)
    s = copy.deepcopy(w.systems[0])
    m = copy.deepcopy(w.model)
    p = copy.deepcopy(w.params[0])
    R = w.R[0].copy()
    for k, v in (model_kw or {}).items():
        setattr(m, k, v)
    if system_fn:
        s, m, p, R = system_fn(s, m, p, R)
    prec = precision or w.precision
    F = fire.Fire(s, m, prec, max_walkers=max(W, 1), **fire_kw)
    F.set_params(p)
    state, ws = F.buffers(W)
    O = Oracle(s, m, p)
    return F, O, s, m, p, R, state, ws


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def small_polyene(W, width=32, n_det=2, n_env=2, ecp=False, seed=7, cutoff=5.0):
    """The C12H14 geometry with a narrow network, so the oracle's autodiff
    Laplacian and full-recompute quadrature stay fast."""
    R, sp = wl.polyene_c12h14()
    rng = np.random.default_rng(seed)
    s = wl.make_system("C12H14", R, sp, pseudo_c=True, nonlocal_ecp=ecp, ecp_rng=rng)
    m = wl.make_model(s, width=width, mlp_layers=2, n_det=n_det, n_env=n_env, cutoff=cutoff, cutoff_nuc=20.0)
    p = wl.init_params(s, m, rng)
    return s, m, p, wl.init_walkers(s, W, rng)


def setup_custom(s, m, p, R, precision, **fire_kw):
    from oracle import Oracle
    from paper_2504_06087_amd import fire
    W = R.shape[0]
    F = fire.Fire(s, m, precision, max_walkers=W, **fire_kw)
    F.set_params(p)
    state, ws = F.buffers(W)
    return F, Oracle(s, m, p), state, ws
