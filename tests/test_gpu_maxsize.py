"""Parity at the large systems: 128 electrons per spin (the cumulene C63H4
with pseudo-carbons, 256 valence electrons, c = 3 bohr), the largest block of
the 16 x 16-thread register inversion; 136 per spin (C67H4, 272 electrons),
past it: the 32 x 32-thread inversion and 512-thread neighbour lists; and 192
per spin (C95H4, 384 electrons), the largest supported.  A narrow network
keeps the oracle's full-recompute chain to about a minute."""
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


def _chain(nc, W, seed, nspin):
    from paper_2504_06087_amd import fire
    rng = np.random.default_rng(seed)
    R, sp = wl.cumulene(nc)
    s = wl.make_system(f"C{nc}H4", R, sp, pseudo_c=True, per_species=True)
    assert s.n_up == nspin and s.n_dn == nspin
    m = wl.make_model(s, width=32, mlp_layers=1, n_det=2, n_env=2, cutoff=3.0, cutoff_nuc=20.0)
    p = wl.init_params(s, m, rng)
    Rw = wl.init_walkers(s, W, rng)
    return s, m, p, Rw, rng


def test_cumulene_136_per_spin_matches_oracle(lib):
    from oracle import Oracle
    from paper_2504_06087_amd import fire
    s, m, p, Rw, rng = _chain(67, 2, 6, 136)
    log("case: C67H4 fp64 W=2 (136 electrons per spin): evaluation and one sweep")
    F = fire.Fire(s, m, "fp64", max_walkers=2, cap_nbr=64, cap_upd=64)
    F.set_params(p)
    state, ws = F.buffers(2)
    O = Oracle(s, m, p)
    Rd = dev(Rw)
    sg, lp, st = F.eval_logpsi(Rd, state, ws)
    torch.cuda.synchronize()
    so, lo = O.log_psi(Rw)
    log(f"log|psi| {lo.numpy()}, err {np.abs(lp.cpu().numpy() - lo.numpy()).max():.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    xi, u = wl.mcmc_noise(1, s.n_el, 2, rng)
    nacc, sg, lp, st = F.mcmc_sweep(Rd, state, ws, 1, 0.2, dev(xi), dev(u))
    torch.cuda.synchronize()
    Ro, so, lo, no = O.mcmc_sweep(Rw, 0.2, xi, u)
    Rg = Rd.cpu().numpy()
    log(f"sweep: accepts {nacc.cpu().numpy()} vs {no.numpy()}, |dR| {np.abs(Rg - Ro.numpy()).max():.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(nacc.cpu().numpy(), no.numpy())
    assert np.abs(Rg - Ro.numpy()).max() <= 1e-12
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-9


def test_cumulene_192_per_spin_evaluation_and_updates(lib):
    """Evaluation against the oracle at the largest supported block; then a
    sweep whose cached inverse and log|psi| must equal a fresh evaluation."""
    from oracle import Oracle
    from paper_2504_06087_amd import fire
    s, m, p, Rw, rng = _chain(95, 2, 7, 192)
    log("case: C95H4 fp64 W=2 (192 electrons per spin): evaluation, sweep vs fresh evaluation")
    F = fire.Fire(s, m, "fp64", max_walkers=2, cap_nbr=64, cap_upd=64)
    F.set_params(p)
    state, ws = F.buffers(2)
    Rd = dev(Rw)
    sg, lp, st = F.eval_logpsi(Rd, state, ws)
    torch.cuda.synchronize()
    so, lo = Oracle(s, m, p).log_psi(Rw)
    log(f"log|psi| {lo.numpy()}, err {np.abs(lp.cpu().numpy() - lo.numpy()).max():.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    xi, u = wl.mcmc_noise(1, s.n_el, 2, rng)
    nacc, sg, lp, st = F.mcmc_sweep(Rd, state, ws, 1, 0.2, dev(xi), dev(u))
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    G1 = F.state_view(state, 2, "inv").clone()
    st2, ws2 = F.buffers(2)
    _, lp2, _ = F.eval_logpsi(Rd, st2, ws2)
    torch.cuda.synchronize()
    eg = float(((G1 - F.state_view(st2, 2, "inv")).abs().max() / F.state_view(st2, 2, "inv").abs().max()).cpu())
    el = float((lp - lp2).abs().max().cpu())
    log(f"accepts {nacc.cpu().numpy()}; cached vs fresh: G {eg:.1e}, log|psi| {el:.1e}")
    assert eg <= 1e-7 and el <= 1e-9


def test_kinetic_energy_matches_finite_differences_136_per_spin(lib):
    """The sparse forward Laplacian past 128 electrons per spin against
    central differences of the library's own FP64 log|psi|: the kinetic energy
    is -1/2 sum_k (d_k^2 log|psi| + (d_k log|psi|)^2) over all 3n coordinates,
    the displaced configurations evaluated as one batch of walkers (h = 1e-3:
    truncation ~h^2, rounding ~1e-16 |log psi| / h^2 per coordinate)."""
    from paper_2504_06087_amd import fire
    s, m, p, Rw, rng = _chain(67, 1, 8, 136)
    R0 = Rw[0]
    n3 = 3 * s.n_el
    h = 1e-3
    batch = np.repeat(R0[None], 1 + 2 * n3, axis=0)
    for k in range(n3):
        batch[1 + 2 * k].reshape(-1)[k] += h
        batch[2 + 2 * k].reshape(-1)[k] -= h
    Wb = batch.shape[0]
    log(f"case: C67H4 fp64, kinetic energy vs central differences over {n3} coordinates ({Wb} evaluations)")
    F = fire.Fire(s, m, "fp64", max_walkers=Wb, cap_nbr=64, cap_upd=64)
    F.set_params(p)
    state, ws = F.buffers(Wb)
    Bd = dev(batch)
    _, lp, st = F.eval_logpsi(Bd, state, ws)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == 0).all()
    f = lp.cpu().numpy()
    fp, fm = f[1::2], f[2::2]
    kin_fd = -0.5 * np.sum((fp - 2 * f[0] + fm) / h ** 2 + ((fp - fm) / (2 * h)) ** 2)
    st1, ws1 = F.buffers(1)
    R1 = dev(R0[None])
    F.eval_logpsi(R1, st1, ws1)
    e, parts, _, st2 = F.local_energy(R1, st1, ws1)
    torch.cuda.synchronize()
    kin = float(parts.cpu().numpy()[0, 0])
    rel = abs(kin - kin_fd) / max(1.0, abs(kin_fd))
    log(f"kinetic {kin:.8f} vs finite differences {kin_fd:.8f}: rel {rel:.1e}")
    assert (st2.cpu().numpy() == 0).all()
    assert rel <= 1e-4
