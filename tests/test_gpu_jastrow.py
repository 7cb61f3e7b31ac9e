"""GPU parity with a non-zero cusp Jastrow factor (Methods, global electron
correlation: J_cusp with learnable w_par, a_par, w_anti, a_anti): log|psi|,
the Metropolis chain (the ratio gains exp(dJ) for the moved electron), the
local energy (grad J, Lap J and the cross term with the determinants), the
nonlocal pseudopotential ratios and the parameter gradient, all against
the FP64 oracle, whose log|psi| includes the factor."""
import copy

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import dev, log, setup, setup_custom, small_polyene

pytestmark = pytest.mark.gpu

JAS = np.array([-0.25, 0.8, -0.5, 1.2])


def _with_jastrow(p):
    p = copy.deepcopy(p)
    p["jas_cusp"] = JAS.copy()
    return p


def test_h4_jastrow_matches_oracle(lib):
    from oracle import Oracle
    log("case: H4 fp64 W=32 with the cusp Jastrow: log|psi|, 5 sweeps, E_L, gradient")
    w = wl.config(0, walkers=32)
    s, m, p, R = w.systems[0], w.model, _with_jastrow(w.params[0]), w.R[0].copy()
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    Rd = dev(R)
    sg, lp, st = F.eval_logpsi(Rd, state, ws)
    torch.cuda.synchronize()
    so, lo = O.log_psi(R)
    assert float(np.abs(O.jastrow_cusp(R).numpy()).min()) > 1e-3
    assert (st.cpu().numpy() == 0).all()
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    rng = np.random.default_rng(9)
    xi, u = wl.mcmc_noise(5, s.n_el, 32, rng)
    nacc, sg, lp, st = F.mcmc_sweep(Rd, state, ws, 5, 0.2, dev(xi), dev(u))
    torch.cuda.synchronize()
    Ro, so, lo, no = O.mcmc_sweep(R, 0.2, xi, u)
    Rg = Rd.cpu().numpy()
    log(f"chain: accepts {int(nacc.sum())} vs {int(no.sum())}, |dR| {np.abs(Rg - Ro.numpy()).max():.1e}, "
        f"|dlogpsi| {np.abs(lp.cpu().numpy() - lo.numpy()).max():.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(nacc.cpu().numpy(), no.numpy())
    assert np.abs(Rg - Ro.numpy()).max() <= 1e-12
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    # the cached log J equals a fresh evaluation at the final positions
    J1 = F.state_view(state, 32, "jas").clone()
    st2, ws2 = F.buffers(32)
    F.eval_logpsi(Rd, st2, ws2)
    torch.cuda.synchronize()
    assert float((J1 - F.state_view(st2, 32, "jas")).abs().max()) <= 1e-12
    e, parts, g, st = F.local_energy(Rd, state, ws, None, want_grad=True)
    torch.cuda.synchronize()
    eo, po = O.local_energy(Rg)
    go, _ = O.grad_lap(Rg)
    err = np.abs(e.cpu().numpy() - eo.numpy()).max()
    log(f"E_L err {err:.1e}; grad log|psi| err {np.abs(g.cpu().numpy() - go.numpy()).max():.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert err <= 1e-8
    assert np.abs(g.cpu().numpy() - go.numpy()).max() <= 1e-9
    coeff = rng.normal(size=32)
    gp, st = F.grad_params(Rd, state, ws, dev(coeff))
    torch.cuda.synchronize()
    ref = F.flatten({k: v.numpy() for k, v in O.grad_params(Rg, coeff).items()})
    gp = gp.cpu().numpy()
    off = [o for name, o, shp in F.layout if name == "jas_cusp"][0]
    log(f"jastrow gradient {gp[off:off + 4]} vs {ref[off:off + 4]}; "
        f"whole vector rel err {np.abs(gp - ref).max() / np.abs(ref).max():.1e}")
    assert np.abs(gp[off:off + 4] - ref[off:off + 4]).max() <= 1e-10 * max(1.0, np.abs(ref[off:off + 4]).max())
    assert np.abs(gp - ref).max() <= 1e-10 * np.abs(ref).max()


def test_polyene_ecp_jastrow_matches_oracle(lib):
    log("case: narrow C12H14 fp64 W=2 with the cusp Jastrow: V_NL and E_L")
    s, m, p, R = small_polyene(2, ecp=True, seed=11)
    p = _with_jastrow(p)
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    Q = wl.haar_rotations(2, np.random.default_rng(5))
    Rd = dev(R)
    _, lp, _ = F.eval_logpsi(Rd, state, ws)
    e, parts, _, st = F.local_energy(Rd, state, ws, dev(Q))
    torch.cuda.synchronize()
    _, lo = O.log_psi(R)
    eo, po = O.local_energy(R, Q, chunk=32)
    vnl_err = np.abs(parts.cpu().numpy()[:, 4] - po.numpy()[:, 4]).max()
    err = (np.abs(e.cpu().numpy() - eo.numpy()) / np.maximum(1.0, np.abs(eo.numpy()))).max()
    log(f"log|psi| err {np.abs(lp.cpu().numpy() - lo.numpy()).max():.1e}; V_NL err {vnl_err:.1e}; "
        f"E_L rel err {err:.1e} (E_L {eo.numpy()})")
    assert (st.cpu().numpy() == 0).all()
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    assert vnl_err <= 1e-9
    assert err <= 1e-8
