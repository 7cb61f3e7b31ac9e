"""Uneven multi-system batches through the C-ABI (fire_batch_*): one step =
evaluation, Metropolis sweep, local energy, energy-gradient coefficients and
the parameter gradient for every system, shared embedding parameters and
per-system orbitals (Methods, wave function ansatz).

* each system in the batch equals the same system run alone;
* in FP64 the batch matches the oracle (its own chain, E_L and gradient);
* a captured graph replays the eager step (the gradient bit for bit);
* the tile autotuner never changes results.
"""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import log

pytestmark = pytest.mark.gpu

STEP = 0.2


def small_batch(W=(6, 4, 5), seed=11, width=32, layers=1, n_det=2, jastrow=False):
    """Three systems of uneven size: H6 chain, a grown C4H4 flake (20
    electrons), H9 chain (odd electron count); with jastrow, the MLP and
    attention Jastrows (shared like the embedding)."""
    rng = np.random.default_rng(seed)
    geoms = [wl.h_chain(6), wl.grown_flake(20), wl.h_chain(9)]
    systems = [wl.make_system(f"b{k}", R, sp, pseudo_c=True, per_species=True) for k, (R, sp) in enumerate(geoms)]
    m = wl.Model(width=width, mlp_layers=layers, n_det=n_det, n_env=2, cutoff=5.0, cutoff_nuc=20.0,
                 n_nuc_types=2)
    if jastrow:
        m.jas_mlp_width, m.jas_att_regs, m.jas_att_dim, m.jas_att_width = 16, 4, 4, 16
    params = [wl.init_params(s, m, rng) for s in systems]
    shared, private = wl.batch_params(params)
    Rs = [wl.init_walkers(s, w, rng) for s, w in zip(systems, W)]
    noise = [wl.mcmc_noise(1, s.n_el, w, rng) for s, w in zip(systems, W)]
    return systems, m, shared, private, Rs, noise


def _batch(lib, precision, split=0, **kw):
    from paper_2504_06087_amd import fire
    systems, m, shared, private, Rs, noise = small_batch(**kw)
    W = [r.shape[0] for r in Rs]
    B = fire.FireBatch(systems, m, precision, W, cap_nbr=48, cap_upd=64, bf16_split=split)
    B.set_params(B.flatten(shared, private))
    R = B.concat(Rs)
    xi = B.concat([x for x, _ in noise])
    u = B.concat([v for _, v in noise])
    state, ws = B.buffers(1)
    nacc = torch.zeros(sum(W), dtype=torch.int32, device="cuda")
    return B, systems, m, shared, private, Rs, noise, R, xi, u, state, ws, nacc


def test_batch_equals_each_system_alone(lib):
    from paper_2504_06087_amd import fire
    log("case: uneven batch (H6, C4H4, H9) fp64 vs each system alone")
    B, systems, m, shared, private, Rs, noise, R, xi, u, state, ws, nacc = _batch(lib, "fp64")
    e, g, st = B.step(R, state, ws, 1, STEP, xi, u, nacc)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    e_b = B.split_walkers(e)
    R_b = B.split_positions(R)
    n_b = B.split_walkers(nacc)
    gsum = None
    for k, s in enumerate(systems):
        W = Rs[k].shape[0]
        F = fire.Fire(s, m, "fp64", max_walkers=W, cap_nbr=min(48, s.n_el - 1), cap_upd=min(64, s.n_el))
        F.set_params(wl.system_params(shared, private[k]))
        st1, ws1 = F.buffers(W)
        Rk = torch.tensor(Rs[k], dtype=torch.float64, device="cuda")
        F.eval_logpsi(Rk, st1, ws1)
        xk = torch.tensor(noise[k][0], device="cuda")
        uk = torch.tensor(noise[k][1], device="cuda")
        na, _, _, _ = F.mcmc_sweep(Rk, st1, ws1, 1, STEP, xk, uk)
        ek, _, _, _ = F.local_energy(Rk, st1, ws1)
        c = (ek - ek.mean()) / W
        gk, _ = F.grad_params(Rk, st1, ws1, c)
        torch.cuda.synchronize()
        assert torch.equal(R_b[k], Rk), k
        assert torch.equal(n_b[k], na), k
        de = float((e_b[k] - ek).abs().max() / ek.abs().max())
        log(f"system {k} (n={s.n_el}, W={W}): E_L rel diff {de:.1e}")
        assert de <= 1e-12
        P0 = B.P_shared
        priv = g[B.priv_off[k]:B.priv_off[k] + gk.numel() - P0]
        dg = float((priv - gk[P0:]).abs().max() / gk.abs().max())
        assert dg <= 1e-10, (k, dg)
        gsum = gk[:P0].clone() if gsum is None else gsum + gk[:P0]
    ds = float((g[:B.P_shared] - gsum).abs().max() / gsum.abs().max())
    log(f"shared gradient = sum over systems: rel diff {ds:.1e}")
    assert ds <= 1e-10


@pytest.mark.parametrize("jastrow", [False, True])
def test_batch_fp64_matches_oracle(lib, jastrow):
    from oracle import Oracle
    log(f"case: uneven batch fp64 vs oracle chain, E_L and summed gradient (neural Jastrows {jastrow})")
    B, systems, m, shared, private, Rs, noise, R, xi, u, state, ws, nacc = _batch(lib, "fp64", jastrow=jastrow)
    e, g, st = B.step(R, state, ws, 1, STEP, xi, u, nacc)
    torch.cuda.synchronize()
    e_b = B.split_walkers(e)
    R_b = B.split_positions(R)
    n_b = B.split_walkers(nacc)
    gsh = None
    for k, s in enumerate(systems):
        O = Oracle(s, m, wl.system_params(shared, private[k]))
        Ro, _, _, no = O.mcmc_sweep(Rs[k], STEP, noise[k][0], noise[k][1])
        assert np.array_equal(n_b[k].cpu().numpy(), no.numpy())
        assert np.abs(R_b[k].cpu().numpy() - Ro.numpy()).max() <= 1e-12
        eo, _ = O.local_energy(Ro)
        eo = eo.numpy()
        de = np.abs(e_b[k].cpu().numpy() - eo).max() / np.abs(eo).max()
        log(f"system {k}: E_L rel diff vs oracle {de:.1e}")
        assert de <= 1e-8
        W = len(eo)
        go = O.grad_params(Ro, (eo - eo.mean()) / W)
        lay = B.layouts[k]
        for name, off, shape in lay:
            ref = go[name].numpy().reshape(-1)
            if off < B.P_shared:
                gsh = {} if gsh is None else gsh
                gsh[name] = gsh.get(name, 0.0) + ref
            else:
                o = B.priv_off[k] + off - B.P_shared
                got = g[o:o + ref.size].cpu().numpy()
                scale = max(np.abs(ref).max(), 1e-300)
                assert np.abs(got - ref).max() / scale <= 1e-8, (k, name)
    worst = 0.0
    for name, off, shape in B.layouts[0]:
        if off < B.P_shared:
            ref = gsh[name]
            got = g[off:off + ref.size].cpu().numpy()
            scale = np.abs(ref).max()
            if scale > 0:
                worst = max(worst, np.abs(got - ref).max() / scale)
    log(f"shared gradient vs oracle sum: worst rel {worst:.1e}")
    assert worst <= 1e-8


def test_graph_replays_match_eager(lib):
    from paper_2504_06087_amd import fire
    log("case: uneven batch bf16 hybrid, graph replay vs eager")
    B, systems, m, shared, private, Rs, noise, R, xi, u, state, ws, nacc = _batch(lib, "bf16", split=7)
    R0 = R.clone()
    e1, g1, st1 = B.step(R, state, ws, 1, STEP, xi, u, nacc)
    torch.cuda.synchronize()
    R1, n1 = R.clone(), nacc.clone()
    out = B.outputs()
    G = B.graph(R, state, ws, 1, STEP, xi, u, nacc, out)
    for rep in range(3):
        R.copy_(R0)
        nacc.zero_()
        torch.cuda.synchronize()
        G.launch()
        torch.cuda.synchronize()
        e2, g2, st2 = out
        assert torch.equal(R, R1), rep
        assert torch.equal(nacc, n1), rep
        assert torch.equal(st2, st1), rep
        de = float((e2 - e1).abs().max() / e1.abs().max())
        dg = float((g2 - g1).abs().max() / g1.abs().max())
        log(f"replay {rep}: E_L rel {de:.1e}, grad rel {dg:.1e}")
        assert de <= 1e-12
        # every reduction of the adjoint has a fixed order
        assert torch.equal(g2, g1), (rep, dg)
        # eager work of the program between replays
        R.copy_(R0)
        nacc.zero_()
        B.step(R, state, ws, 1, STEP, xi, u, nacc)
        torch.cuda.synchronize()
        assert torch.equal(R, R1)


def test_autotuner_keeps_results(lib):
    from paper_2504_06087_amd import fire
    log("case: uneven batch bf16 hybrid, autotuned tiles vs default tiles")
    B, systems, m, shared, private, Rs, noise, R, xi, u, state, ws, nacc = _batch(lib, "bf16", split=7)
    R0 = R.clone()
    fire.autotune_clear()
    e1, g1, _ = B.step(R, state, ws, 1, STEP, xi, u, nacc)
    torch.cuda.synchronize()
    R1 = R.clone()
    fire.autotune(True)
    try:
        R.copy_(R0)
        et, gt, _ = B.step(R, state, ws, 1, STEP, xi, u, nacc)
        torch.cuda.synchronize()
    finally:
        fire.autotune(False)
    # the timing launches rewrite GEMM outputs with the same values
    assert torch.equal(R, R1)
    assert float((et - e1).abs().max() / e1.abs().max()) <= 1e-12
    n = fire.autotune_count()
    log(f"tuned shapes: {n}")
    assert n > 0
    R.copy_(R0)
    e2, g2, _ = B.step(R, state, ws, 1, STEP, xi, u, nacc)
    torch.cuda.synchronize()
    assert torch.equal(R, R1)
    assert float((e2 - e1).abs().max() / e1.abs().max()) <= 1e-12
    assert torch.equal(g2, g1)
    fire.autotune_clear()


def test_graph_with_nonlocal_channels_matches_eager(lib):
    """A batch whose system has nonlocal channels captures too (the
    quadrature reads its job counts on the device): three replays with eager
    steps between them equal the eager step."""
    from paper_2504_06087_amd import fire
    log("case: uneven batch with nonlocal channels fp64: graph replay vs eager")
    rng = np.random.default_rng(5)
    R, sp = wl.grown_flake(20)
    s = wl.make_system("ecp", R, sp, pseudo_c=True, per_species=True, nonlocal_ecp=True, ecp_rng=rng)
    m = wl.Model(width=32, mlp_layers=1, n_det=2, n_env=2, n_nuc_types=2)
    p = wl.init_params(s, m, rng)
    shared, private = wl.batch_params([p])
    B = fire.FireBatch([s], m, "fp64", [2])
    B.set_params(B.flatten(shared, private))
    Rd = B.concat([wl.init_walkers(s, 2, rng)])
    state, ws = B.buffers(0)
    e1, g1, st1 = B.step(Rd, state, ws, 0, STEP, None, None, None)
    torch.cuda.synchronize()
    e1, g1, st1 = e1.clone(), g1.clone(), st1.clone()
    out = B.outputs()
    G = B.graph(Rd, state, ws, 0, STEP, None, None, None, out)
    for rep in range(3):
        out[0].zero_()
        G.launch()
        torch.cuda.synchronize()
        e2, g2, st2 = out
        de = float((e2 - e1).abs().max())
        dg = float((g2 - g1).abs().max() / g1.abs().max())
        log(f"replay {rep}: E_L {e2.cpu().numpy()} vs eager {e1.cpu().numpy()}; grad rel {dg:.1e}")
        assert torch.equal(st2, st1) and int(st2.abs().sum()) == 0
        assert de <= 1e-12 * float(e1.abs().max())
        assert dg <= 1e-12
        B.step(Rd, state, ws, 0, STEP, None, None, None)
        torch.cuda.synchronize()
