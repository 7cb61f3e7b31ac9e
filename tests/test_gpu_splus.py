"""GPU parity of fire_splus_ratios, the two-electron swap ratios of the S+
spin penalty computed by low-rank updates (SI, low-rank updates in S+
operator), against the oracle's full re-evaluation of every swapped
configuration."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import dev, log, setup, setup_custom, small_polyene

pytestmark = pytest.mark.gpu


def _gpu(F, R, state, ws, beta):
    Rd = dev(R)
    F.eval_logpsi(Rd, state, ws)
    r, rb, st = F.splus_ratios(Rd, state, ws, beta)
    torch.cuda.synchronize()
    return r.cpu().numpy(), rb.cpu().numpy(), st.cpu().numpy()


def _check(F, O, R, state, ws, beta, tol, tag):
    r, rb, st = _gpu(F, R, state, ws, beta)
    ro, rbo = O.splus_ratios(R, beta)
    ro, rbo = ro.numpy(), rbo.numpy()
    err = np.abs(r - ro).max() / max(1.0, np.abs(ro).max())
    log(f"{tag}: beta={beta} max ratio err {err:.1e}; R_beta gpu {rb[:3]} oracle {rbo[:3]}")
    assert (st == 0).all()
    assert err <= tol
    assert np.abs(rb - rbo).max() <= tol * max(1.0, np.abs(rbo).max()) * r.shape[1]


@pytest.mark.parametrize("beta", [2, 3])
def test_h4_swap_ratios(lib, beta):
    log("case: H4 fp64 W=16 S+ swap ratios")
    F, O, s, m, p, R, state, ws = setup(0, 16, "fp64")
    _check(F, O, R, state, ws, beta, 1e-10, "H4")


def test_h4_swap_ratios_with_cusp_jastrow(lib):
    def jas(s, m, p, R):
        p["jas_cusp"] = np.array([-0.25, 0.8, -0.5, 1.2])
        return s, m, p, R
    F, O, s, m, p, R, state, ws = setup(0, 8, "fp64", system_fn=jas)
    _check(F, O, R, state, ws, 2, 1e-10, "H4 + cusp Jastrow")


def test_closed_shell_penalty_vanishes_on_gpu(lib):
    """Zeroed network and one set of spatial orbitals for both spins: R_beta =
    0 at every walker (the oracle pin's identity, here through the low-rank
    path)."""
    w = wl.config(0, walkers=8)
    s, m = w.systems[0], w.model
    m.n_det = 2
    p = wl.init_params(s, m, np.random.default_rng(4))
    wl.zero_network(p)
    p["orb_W_dn"] = p["orb_W_up"].copy()
    p["env_pi_dn"] = p["env_pi_up"].copy()
    F, O, state, ws = setup_custom(s, m, p, w.R[0], "fp64")
    r, rb, st = _gpu(F, w.R[0], state, ws, 3)
    log(f"closed shell: max |R_beta| {np.abs(rb).max():.1e}")
    assert (st == 0).all() and np.abs(rb).max() <= 1e-10


@pytest.mark.parametrize("cutoff", [5.0, 1e-9])
def test_polyene_swap_ratios(lib, cutoff):
    """31 + 31 electrons, narrow network: update sets of the two positions'
    neighbourhoods (c = 5) and the two moved electrons alone (c -> 0)."""
    log(f"case: narrow C12H14 fp64 W=2 S+ swap ratios c={cutoff}")
    s, m, p, R = small_polyene(2, cutoff=cutoff, seed=3)
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    _check(F, O, R, state, ws, 40, 1e-9, "C12H14")


def test_benchnet_swap_ratios(lib):
    """The benchmark's network (width 256, 3 layers, 16 determinants) on the
    20-electron flake."""
    log("case: C4H4 benchmark network fp64 W=2 S+ swap ratios")
    rng = np.random.default_rng(31)
    Rg, sp = wl.grown_flake(20)
    s = wl.make_system("C4H4", Rg, sp, pseudo_c=True)
    m = wl.make_model(s, width=256, mlp_layers=3, n_det=16, n_env=8, cutoff=5.0, cutoff_nuc=20.0)
    p = wl.init_params(s, m, rng)
    R = wl.init_walkers(s, 2, rng)
    F, O, state, ws = setup_custom(s, m, p, R, "fp64", cap_nbr=48, cap_upd=64)
    _check(F, O, R, state, ws, 13, 1e-9, "C4H4 benchmark network")


def test_swap_argument_errors(lib):
    from paper_2504_06087_amd import fire
    F, O, s, m, p, R, state, ws = setup(0, 2, "fp64")
    Rd = dev(R)
    F.eval_logpsi(Rd, state, ws)
    for beta in (0, 1, 4):
        with pytest.raises(fire.FireError):
            F.splus_ratios(Rd, state, ws, beta)
