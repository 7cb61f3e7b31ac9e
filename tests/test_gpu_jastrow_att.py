"""GPU parity with the attention-register Jastrow factor (Methods, global
electron correlation: registers v_r = softmax_i(h_i . q_r)^T (h_i W^V_r) and
J_att = exp(MLP_1(V)) MLP_2(V)), alone and beside the MLP Jastrow, against
the FP64 oracle: log|psi| and its sign, the Metropolis chain (the update
rows change the cached softmax sums), cached against fresh sums, the local
energy (dense tangents of the registers through the readout MLPs), the
nonlocal pseudopotential ratios, the S+ swap ratios and the parameter
gradient including the queries, value maps and readouts."""
import copy

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import dev, log, setup_custom, small_polyene

pytestmark = pytest.mark.gpu


def _h4(W, b3_node, with_mlp, seed=23):
    w = wl.config(0, walkers=W)
    s, m, R = w.systems[0], copy.deepcopy(w.model), w.R[0].copy()
    m.jas_att_regs, m.jas_att_dim, m.jas_att_width = 4, 4, 16
    m.jas_mlp_width = 16 if with_mlp else 0
    p = wl.init_params(s, m, np.random.default_rng(seed))
    p["jatt_b3"] = np.array([0.2, b3_node])
    return s, m, p, R


@pytest.mark.parametrize("b3_node,with_mlp", [(1.0, False), (-1.0, True)])
def test_h4_att_jastrow_matches_oracle(lib, b3_node, with_mlp):
    W = 32
    log(f"case: H4 fp64 W={W} attention Jastrow (node bias {b3_node}, MLP Jastrow {with_mlp}): "
        "log|psi|, 5 sweeps, E_L, gradient")
    s, m, p, R = _h4(W, b3_node, with_mlp)
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    Rd = dev(R)
    sg, lp, st = F.eval_logpsi(Rd, state, ws)
    torch.cuda.synchronize()
    so, lo = O.log_psi(R)
    log(f"log|psi| err {np.abs(lp.cpu().numpy() - lo.numpy()).max():.1e}; signs "
        f"{sg.cpu().numpy()[:6]} vs {so.numpy()[:6]}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    rng = np.random.default_rng(9)
    xi, u = wl.mcmc_noise(5, s.n_el, W, rng)
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
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    J1 = F.state_view(state, W, "jas").clone()
    st2, ws2 = F.buffers(W)
    F.eval_logpsi(Rd, st2, ws2)
    torch.cuda.synchronize()
    dj = float((J1 - F.state_view(st2, W, "jas")).abs().max())
    log(f"cached vs fresh Jastrow log: {dj:.1e}")
    assert dj <= 1e-11
    e, parts, g, st = F.local_energy(Rd, state, ws, None, want_grad=True)
    torch.cuda.synchronize()
    eo, po = O.local_energy(Rg)
    go, _ = O.grad_lap(Rg)
    err = (np.abs(e.cpu().numpy() - eo.numpy()) / np.maximum(1.0, np.abs(eo.numpy()))).max()
    gerr = np.abs(g.cpu().numpy() - go.numpy()).max()
    log(f"E_L rel err {err:.1e}; grad log|psi| err {gerr:.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert err <= 1e-8
    assert gerr <= 1e-9
    coeff = rng.normal(size=W)
    gp, st = F.grad_params(Rd, state, ws, dev(coeff))
    torch.cuda.synchronize()
    ref = F.flatten({k: v.numpy() for k, v in O.grad_params(Rg, coeff).items()})
    gp = gp.cpu().numpy()
    for name, off, shp in F.layout:
        if name.startswith("jatt_") or name.startswith("jmlp_"):
            sz = int(np.prod(shp))
            e_ = np.abs(gp[off:off + sz] - ref[off:off + sz]).max() / max(1e-300, np.abs(ref[off:off + sz]).max())
            log(f"  {name}: rel err {e_:.1e}")
            assert e_ <= 1e-10
    rel = np.abs(gp - ref).max() / np.abs(ref).max()
    log(f"whole gradient rel err {rel:.1e}")
    assert rel <= 1e-10


def test_polyene_ecp_att_jastrow_matches_oracle(lib):
    log("case: narrow C12H14 fp64 W=2 with both neural Jastrows: log|psi|, V_NL, E_L, gradient")
    s, m, p, R = small_polyene(2, ecp=True, seed=11)
    m = copy.deepcopy(m)
    m.jas_mlp_width = 16
    m.jas_att_regs, m.jas_att_dim, m.jas_att_width = 4, 4, 16
    p = wl.init_params(s, m, np.random.default_rng(37))
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    Q = wl.haar_rotations(2, np.random.default_rng(5))
    Rd = dev(R)
    sg, lp, _ = F.eval_logpsi(Rd, state, ws)
    e, parts, _, st = F.local_energy(Rd, state, ws, dev(Q))
    torch.cuda.synchronize()
    so, lo = O.log_psi(R)
    eo, po = O.local_energy(R, Q, chunk=32)
    vnl_err = np.abs(parts.cpu().numpy()[:, 4] - po.numpy()[:, 4]).max()
    kin_err = np.abs(parts.cpu().numpy()[:, 0] - po.numpy()[:, 0]).max() / max(1.0, np.abs(po.numpy()[:, 0]).max())
    err = (np.abs(e.cpu().numpy() - eo.numpy()) / np.maximum(1.0, np.abs(eo.numpy()))).max()
    log(f"log|psi| err {np.abs(lp.cpu().numpy() - lo.numpy()).max():.1e}; kinetic rel err {kin_err:.1e}; "
        f"V_NL err {vnl_err:.1e}; E_L rel err {err:.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    assert vnl_err <= 1e-9
    assert err <= 1e-8
    coeff = np.array([0.6, -1.1])
    gp, st = F.grad_params(Rd, state, ws, dev(coeff))
    torch.cuda.synchronize()
    ref = F.flatten({k: v.numpy() for k, v in O.grad_params(R, coeff).items()})
    rel = np.abs(gp.cpu().numpy() - ref).max() / np.abs(ref).max()
    log(f"gradient rel err {rel:.1e}")
    assert rel <= 1e-10


def test_h4_att_jastrow_swap_ratios(lib):
    log("case: H4 fp64 W=8 with the attention Jastrow: S+ swap ratios")
    s, m, p, R = _h4(8, -1.0, False)
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    Rd = dev(R)
    F.eval_logpsi(Rd, state, ws)
    for beta in (2, 3):
        r, rb, st = F.splus_ratios(Rd, state, ws, beta)
        torch.cuda.synchronize()
        ro, rbo = O.splus_ratios(R, beta)
        err = np.abs(r.cpu().numpy() - ro.numpy()).max() / max(1.0, np.abs(ro.numpy()).max())
        log(f"beta={beta}: ratio err {err:.1e}")
        assert (st.cpu().numpy() == 0).all()
        assert err <= 1e-10
        assert np.abs(rb.cpu().numpy() - rbo.numpy()).max() <= 1e-9


@pytest.mark.parametrize("prec,tol_lp,tol_e", [("fp32", 1e-4, 1e-3), ("bf16", 1e-2, 5e-2)])
def test_h4_neural_jastrows_reduced_precision(lib, prec, tol_lp, tol_e):
    """Both neural Jastrows in FP32 and in the BF16 hybrid (split-bf16 GEMMs
    on every site): log|psi| after a sweep and E_L against the FP64 oracle,
    within the precision's rounding (relative to max(1, |value|))."""
    W = 16
    log(f"case: H4 {prec} W={W} with both neural Jastrows: log|psi|, 2 sweeps, E_L")
    s, m, p, R = _h4(W, 1.0, True)
    F, O, state, ws = setup_custom(s, m, p, R, prec, **({"bf16_split": 7} if prec == "bf16" else {}))
    Rd = dev(R)
    sg, lp, st = F.eval_logpsi(Rd, state, ws)
    torch.cuda.synchronize()
    so, lo = O.log_psi(R)
    elp = (np.abs(lp.cpu().numpy() - lo.numpy()) / np.maximum(1.0, np.abs(lo.numpy()))).max()
    rng = np.random.default_rng(4)
    xi, u = wl.mcmc_noise(2, s.n_el, W, rng)
    F.mcmc_sweep(Rd, state, ws, 2, 0.2, dev(xi), dev(u))
    e, parts, _, st2 = F.local_energy(Rd, state, ws, None)
    torch.cuda.synchronize()
    Rg = Rd.cpu().numpy()
    eo, _ = O.local_energy(Rg)
    _, lo2 = O.log_psi(Rg)
    F2, _, s3, w3 = setup_custom(s, m, p, Rg, prec, **({"bf16_split": 7} if prec == "bf16" else {}))
    _, lp2, _ = F2.eval_logpsi(dev(Rg), s3, w3)
    torch.cuda.synchronize()
    elp2 = (np.abs(lp2.cpu().numpy() - lo2.numpy()) / np.maximum(1.0, np.abs(lo2.numpy()))).max()
    ee = (np.abs(e.cpu().numpy() - eo.numpy()) / np.maximum(1.0, np.abs(eo.numpy()))).max()
    log(f"log|psi| rel err {elp:.1e} (after the sweeps {elp2:.1e}); E_L rel err {ee:.1e}")
    assert (st.cpu().numpy() == 0).all() and (st2.cpu().numpy() == 0).all()
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    assert elp <= tol_lp and elp2 <= tol_lp
    assert ee <= tol_e


def test_h4_neural_jastrows_per_walker_gradients(lib):
    """The per-walker gradients (the rows SPRING consumes) with both neural
    Jastrows, against the oracle's one reverse pass per walker."""
    from oracle import per_walker_gradients
    W = 6
    log(f"case: H4 fp64 W={W} with both neural Jastrows: per-walker gradients")
    s, m, p, R = _h4(W, -1.0, True)
    F, O_, state, ws = setup_custom(s, m, p, R, "fp64")
    Rd = dev(R)
    F.eval_logpsi(Rd, state, ws)
    O = torch.empty(W, F.P, dtype=torch.float64, device="cuda")
    coeff = np.random.default_rng(5).normal(size=W)
    g, st = F.grad_params(Rd, state, ws, dev(coeff), per_walker=O)
    torch.cuda.synchronize()
    names = [x[0] for x in F.layout]
    ref = per_walker_gradients(O_, R, names)
    err = np.abs(O.cpu().numpy() - ref).max() / np.abs(ref).max()
    log(f"per-walker rows: max |dO| / max |O| = {err:.1e}")
    assert (st.cpu().numpy() == 0).all()
    assert err <= 1e-10


def test_single_electron_with_neural_jastrows(lib):
    """Edge case: one electron (hydrogen, no spin-down block, no
    neighbours): the softmax runs over a single electron and the jets have
    only the electron's own rows; log|psi|, a sweep, E_L and the gradient
    against the oracle."""
    W = 8
    log(f"case: hydrogen fp64 W={W} with both neural Jastrows")
    s, m, p, R = wl.hydrogen_atom(W=W, seed=3)
    m = copy.deepcopy(m)
    m.jas_mlp_width = 8          # at most the embedding width (8)
    m.jas_att_regs, m.jas_att_dim, m.jas_att_width = 2, 4, 8
    p = wl.init_params(s, m, np.random.default_rng(17))
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    Rd = dev(R)
    sg, lp, st = F.eval_logpsi(Rd, state, ws)
    torch.cuda.synchronize()
    so, lo = O.log_psi(R)
    assert (st.cpu().numpy() == 0).all()
    assert np.array_equal(sg.cpu().numpy(), so.numpy())
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    rng = np.random.default_rng(2)
    xi, u = wl.mcmc_noise(3, s.n_el, W, rng)
    nacc, sg, lp, st = F.mcmc_sweep(Rd, state, ws, 3, 0.3, dev(xi), dev(u))
    torch.cuda.synchronize()
    Ro, so, lo, no = O.mcmc_sweep(R, 0.3, xi, u)
    assert np.array_equal(nacc.cpu().numpy(), no.numpy())
    assert np.abs(Rd.cpu().numpy() - Ro.numpy()).max() <= 1e-12
    assert np.abs(lp.cpu().numpy() - lo.numpy()).max() <= 1e-10
    Rg = Rd.cpu().numpy()
    e, _, _, st = F.local_energy(Rd, state, ws, None)
    coeff = rng.normal(size=W)
    gp, st2 = F.grad_params(Rd, state, ws, dev(coeff))
    torch.cuda.synchronize()
    eo, _ = O.local_energy(Rg)
    ref = F.flatten({k: v.numpy() for k, v in O.grad_params(Rg, coeff).items()})
    ee = (np.abs(e.cpu().numpy() - eo.numpy()) / np.maximum(1.0, np.abs(eo.numpy()))).max()
    eg = np.abs(gp.cpu().numpy() - ref).max() / np.abs(ref).max()
    log(f"E_L rel err {ee:.1e}; gradient rel err {eg:.1e}")
    assert (st.cpu().numpy() == 0).all() and (st2.cpu().numpy() == 0).all()
    assert ee <= 1e-8
    assert eg <= 1e-10
