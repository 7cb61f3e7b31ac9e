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
