"""Parity at the largest supported system: 128 electrons per spin (the
cumulene C63H4 with pseudo-carbons, 256 valence electrons, c = 3 bohr), where
the FP64 Gauss-Jordan block fills 132 KB of LDS and the update kernels run
their largest orbital blocks.  A narrow network keeps the oracle's
full-recompute chain to about a minute."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import dev, log

pytestmark = pytest.mark.gpu


def test_cumulene_128_per_spin_matches_oracle(lib):
    from oracle import Oracle
    from paper_2504_06087_amd import fire
    rng = np.random.default_rng(5)
    R, sp = wl.cumulene(63)
    s = wl.make_system("C63H4", R, sp, pseudo_c=True, per_species=True)
    assert s.n_up == 128 and s.n_dn == 128
    m = wl.make_model(s, width=32, mlp_layers=1, n_det=2, n_env=2, cutoff=3.0, cutoff_nuc=20.0)
    p = wl.init_params(s, m, rng)
    W = 2
    Rw = wl.init_walkers(s, W, rng)
    log("case: C63H4 fp64 W=2 (128 electrons per spin): evaluation and one sweep")
    F = fire.Fire(s, m, "fp64", max_walkers=W, cap_nbr=64, cap_upd=64)
    F.set_params(p)
    state, ws = F.buffers(W)
    O = Oracle(s, m, p)
    Rd = dev(Rw)
    sg, lp, st = F.eval_logpsi(Rd, state, ws)
    torch.cuda.synchronize()
    so, lo = O.log_psi(Rw)
    log(f"log|psi| {lo.numpy()}, err {np.abs(lp.cpu().numpy() - lo.numpy()).max():.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    xi, u = wl.mcmc_noise(1, s.n_el, W, rng)
    nacc, sg, lp, st = F.mcmc_sweep(Rd, state, ws, 1, 0.2, dev(xi), dev(u))
    torch.cuda.synchronize()
    Ro, so, lo, no = O.mcmc_sweep(Rw, 0.2, xi, u)
    Rg = Rd.cpu().numpy()
    log(f"sweep: accepts {nacc.cpu().numpy()} vs {no.numpy()}, |dR| {np.abs(Rg - Ro.numpy()).max():.1e}, "
        f"|dlogpsi| {np.abs(lp.cpu().numpy() - lo.numpy()).max():.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(nacc.cpu().numpy(), no.numpy())
    assert np.abs(Rg - Ro.numpy()).max() <= 1e-12
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-9
    # cached state vs a fresh evaluation at the final positions
    G1 = F.state_view(state, W, "inv").clone()
    L1 = F.state_view(state, W, "lpsi").clone()
    st2, ws2 = F.buffers(W)
    F.eval_logpsi(Rd, st2, ws2)
    torch.cuda.synchronize()
    G2 = F.state_view(st2, W, "inv")
    eg = float(((G1 - G2).abs().max() / G2.abs().max()).cpu())
    el = float((L1 - F.state_view(st2, W, "lpsi")).abs().max().cpu())
    log(f"cached vs fresh: G {eg:.1e}, log|det sum| {el:.1e}")
    assert eg <= 1e-7 and el <= 1e-9
