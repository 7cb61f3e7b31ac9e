"""GPU parity of the per-walker gradients (fire_grad_params with per_walker)
and of the natural-gradient step fire_spring_step (Methods, variational Monte
Carlo, eq. spring; SI, non-hermitian operator gradients in Spring, eq.
aux_spring) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import dev, log, setup, setup_custom

pytestmark = pytest.mark.gpu


def _per_walker(F, R, state, ws, coeff):
    Rd = dev(R)
    F.eval_logpsi(Rd, state, ws)
    O = torch.empty(R.shape[0], F.P, dtype=torch.float64, device="cuda")
    g, st = F.grad_params(Rd, state, ws, dev(coeff), per_walker=O)
    torch.cuda.synchronize()
    return O.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()


def test_h4_per_walker_gradients_match_oracle(lib):
    from oracle import per_walker_gradients
    log("case: H4 fp64 W=6 per-walker gradients")
    F, O_, s, m, p, R, state, ws = setup(0, 6, "fp64")
    coeff = np.random.default_rng(5).normal(size=6)
    O, g, st = _per_walker(F, R[:6], state, ws, coeff)
    names = [x[0] for x in F.layout]
    ref = per_walker_gradients(O_, R[:6], names)
    err = np.abs(O - ref).max() / np.abs(ref).max()
    log(f"per-walker rows: max |dO| / max |O| = {err:.1e}")
    assert (st == 0).all()
    assert err <= 1e-10
    assert np.abs(g - coeff @ ref).max() <= 1e-10 * np.abs(coeff @ ref).max()
    # the batched adjoint gives the same weighted sum
    gb, _ = F.grad_params(dev(R[:6]), state, ws, dev(coeff))
    torch.cuda.synchronize()
    assert np.abs(gb.cpu().numpy() - g).max() <= 1e-11 * np.abs(g).max()


def test_benchnet_per_walker_gradients_match_oracle(lib):
    """The benchmark's network (width 256, 3 layers, 16 determinants) on the
    20-electron flake with nonlocal channels, two walkers."""
    from oracle import per_walker_gradients
    log("case: C4H4 benchmark network fp64 per-walker gradients, W=2")
    rng = np.random.default_rng(31)
    Rg, sp = wl.grown_flake(20)
    s = wl.make_system("C4H4", Rg, sp, pseudo_c=True, nonlocal_ecp=True, ecp_rng=rng)
    m = wl.make_model(s, width=256, mlp_layers=3, n_det=16, n_env=8, cutoff=5.0, cutoff_nuc=20.0)
    p = wl.init_params(s, m, rng)
    R = wl.init_walkers(s, 2, rng)
    F, O_, state, ws = setup_custom(s, m, p, R, "fp64", cap_nbr=48, cap_upd=64)
    O, g, st = _per_walker(F, R, state, ws, np.array([1.0, -0.5]))
    ref = per_walker_gradients(O_, R, [x[0] for x in F.layout])
    err = np.abs(O - ref).max() / np.abs(ref).max()
    log(f"benchmark network per-walker rows: max |dO| / max |O| = {err:.1e}")
    assert (st == 0).all()
    assert err <= 1e-9


@pytest.mark.parametrize("extra", [False, True])
def test_spring_step_matches_oracle(lib, extra):
    """Random per-walker gradients (150 walkers: two full Cholesky blocks of
    64 and a ragged one; the H4 network's parameter count), momentum 0.99,
    damping 1e-3, and optionally an extra gradient split by the damped
    pseudo-inverse."""
    from oracle import spring_step
    log(f"case: spring step W=150 extra={extra}")
    F, *_ = setup(0, 2, "fp64")
    rng = np.random.default_rng(11)
    W, P = 150, F.P
    O = rng.normal(size=(W, P)) + 0.2 * rng.normal(size=P)
    e = rng.normal(size=W) * 3.0 - 2.0
    dprev = 0.05 * rng.normal(size=P)
    dt = 0.1 * rng.normal(size=P) if extra else None
    from paper_2504_06087_amd import fire
    Fw = fire.Fire(F.system, F.model, "fp64", max_walkers=W)
    _, _, wsb = Fw.sizes(W)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    delta, info = Fw.spring_step(dev(O), dev(e), ws, 1e-3, 0.99, dev(dprev), None if dt is None else dev(dt), 1e-9)
    torch.cuda.synchronize()
    ref = spring_step(O, e, 1e-3, 0.99, dprev, dt, 1e-9)
    err = np.abs(delta.cpu().numpy() - ref).max() / np.abs(ref).max()
    log(f"spring delta: max rel err {err:.1e} (P = {P})")
    assert int(info.item()) == 0
    assert err <= 1e-9


def test_spring_step_end_to_end_h4(lib):
    """One natural-gradient step on H4 from the library's own per-walker
    gradients and local energies against the oracle's."""
    from oracle import per_walker_gradients, spring_step
    log("case: H4 fp64 W=24: per-walker gradients + local energies + spring step")
    F, O_, s, m, p, R, state, ws = setup(0, 24, "fp64")
    R = R[:24]
    O, _, st = _per_walker(F, R, state, ws, np.zeros(24))
    e, _, _, st2 = F.local_energy(dev(R), state, ws)
    delta, info = F.spring_step(torch.tensor(O, device="cuda"), e, ws, 1e-3, 0.99)
    torch.cuda.synchronize()
    eo, _ = O_.local_energy(R)
    ref = spring_step(per_walker_gradients(O_, R, [x[0] for x in F.layout]), eo.numpy(), 1e-3, 0.99)
    err = np.abs(delta.cpu().numpy() - ref).max() / np.abs(ref).max()
    log(f"end-to-end spring delta: max rel err {err:.1e}")
    assert (st == 0).all() and (st2.cpu().numpy() == 0).all() and int(info.item()) == 0
    assert err <= 1e-8
