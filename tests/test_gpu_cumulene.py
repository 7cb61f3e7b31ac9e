"""GPU parity on the cumulene chains of the runtime-scaling study (Fig. 2:
c = 3 bohr, nonlocal pseudopotential on C, element-shared nuclear
parameters): full evaluation, a Metropolis sweep of low-rank updates and the
local energy against the FP64 oracle.  Butatriene (C4H4, coplanar ends) and
pentatetraene (C5H4, perpendicular ends), a narrow network so the oracle's
autodiff Laplacian stays fast."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import dev, log, setup_custom

pytestmark = pytest.mark.gpu


def _cumulene(nc, W, seed):
    rng = np.random.default_rng(seed)
    R, sp = wl.cumulene(nc)
    s = wl.make_system(f"C{nc}H4", R, sp, pseudo_c=True, nonlocal_ecp=True, ecp_rng=rng, per_species=True)
    m = wl.make_model(s, width=32, mlp_layers=2, n_det=2, n_env=2, cutoff=3.0, cutoff_nuc=20.0)
    p = wl.init_params(s, m, rng)
    return s, m, p, wl.init_walkers(s, W, rng), rng


@pytest.mark.parametrize("nc", [4, 5])
def test_cumulene_fp64_matches_oracle(lib, nc):
    W = 3
    log(f"case: C{nc}H4 fp64 c=3 W={W}: eval, 1 sweep, E_L with nonlocal ECP")
    s, m, p, R, rng = _cumulene(nc, W, 40 + nc)
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    Rd = dev(R)
    sg, lp, st = F.eval_logpsi(Rd, state, ws)
    torch.cuda.synchronize()
    so, lo = O.log_psi(R)
    log(f"log|psi| err {np.abs(lp.cpu().numpy() - lo.numpy()).max():.2e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    xi, u = wl.mcmc_noise(1, s.n_el, W, rng)
    nacc, sg, lp, st = F.mcmc_sweep(Rd, state, ws, 1, 0.2, dev(xi), dev(u))
    torch.cuda.synchronize()
    Ro, so, lo, no = O.mcmc_sweep(R, 0.2, xi, u)
    Rg = Rd.cpu().numpy()
    log(f"sweep: accepts {nacc.cpu().numpy()} vs {no.numpy()}, |dR| {np.abs(Rg - Ro.numpy()).max():.2e}, "
        f"|dlogpsi| {np.abs(lp.cpu().numpy() - lo.numpy()).max():.2e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(nacc.cpu().numpy(), no.numpy())
    assert np.abs(Rg - Ro.numpy()).max() <= 1e-12
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    Q = wl.haar_rotations(W, rng)
    e, parts, _, st = F.local_energy(Rd, state, ws, dev(Q))
    torch.cuda.synchronize()
    eo, po = O.local_energy(Rg, Q, chunk=32)
    err = np.abs(e.cpu().numpy() - eo.numpy()).max()
    log(f"E_L err {err:.2e}; V_NL err {np.abs(parts.cpu().numpy()[:, 4] - po.numpy()[:, 4]).max():.2e}")
    assert (st.cpu().numpy() == 0).all()
    assert err <= 1e-7
    assert np.abs(parts.cpu().numpy()[:, 4] - po.numpy()[:, 4]).max() <= 1e-9
