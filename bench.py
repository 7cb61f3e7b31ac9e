"""Throughput of the FiRE hot path on one MI355X.

One step = one pass of the whole hot path over one batch of walkers of the
180-electron C42H12 flake (4096 walkers, width 256, 3 layers, 16
determinants, c = 5 bohr, nonlocal pseudopotential on C):
  full evaluation of log|psi| (neighbours, embeddings, orbitals, FP64 LU),
  one Metropolis sweep of single-electron moves by low-rank updates,
  the local energy (sparse forward Laplacian, potential, nonlocal
  pseudopotential quadrature by low-rank ratios),
  the parameter gradient of sum_w c_w log|psi_w| (when available).
The BF16/FP64-hybrid path is timed, then the same step in plain FP32.

Prints one JSON line.  Inputs are seeded synthetic data resident in HBM when
the timed region starts.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "local energies/s + MCMC walker-steps/s @180 e⁻, BF16-hybrid vs FP32 plain"
HBM_PEAK = 8.0e12
PEAK = {"bf16": 2.5e15, "bf16x3": 2.5e15, "f32": 157.3e12, "f64": 78.6e12}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_traffic_flake180_w4096.txt")
GEMM_SOURCE = os.path.join(ROOT, "paper_2504_06087_amd", "csrc", "gemm.hip")


def measured_traffic():
    """HBM bytes per split-bf16 GEMM launch from the committed counter
    summary, or None when the GEMM source has changed since it was taken."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        src = hashlib.sha256(open(GEMM_SOURCE, "rb").read()).hexdigest()
        if kv.get("gemm_source_sha256") != src:
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def copy_probe():
    import torch
    n = 256 * 1024 * 1024
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_per_copy": n * 4, "copies": 3}))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--walkers", type=int, default=4096)
    ap.add_argument("--split", type=int, default=7, help="split-bf16 GEMM sites of the hybrid precision")
    ap.add_argument("--no-fp32", action="store_true", help="skip the FP32-plain comparison")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-grad", action="store_true")
    ap.add_argument("--no-c5", action="store_true", help="skip the uneven 16-system batch")
    ap.add_argument("--jastrow", action="store_true",
                    help="also time the hybrid step with the MLP and attention Jastrows at the paper's widths")
    ap.add_argument("--no-rule4", action="store_true",
                    help="skip the E_L phase timed with the 4-point pseudopotential rule on C")
    ap.add_argument("--c5-walkers", type=int, default=512)
    ap.add_argument("--scaling", action="store_true",
                    help="runtime-scaling sweep over cumulene chains instead of the step benchmark")
    ap.add_argument("--scaling-carbons", type=str, default="4,8,16,24,32,44,63,80,95",
                    help="chain lengths (carbons); 63 gives 256 electrons, 128 per spin, the largest supported")
    ap.add_argument("--scaling-cutoff", type=float, default=3.0)
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 1 GiB three times (HBM counter calibration under rocprofv3 --pmc)")
    return ap.parse_args()


def run_precision(prec, split, W, steps, warmup, want_grad, profile, jastrow=False):
    import copy
    import torch
    import workloads as wl
    from paper_2504_06087_amd import fire

    work = wl.config(3, walkers=W)
    s, m, p, R0 = work.systems[0], work.model, work.params[0], work.R[0]
    if jastrow:
        # the paper's Jastrow widths: per-electron MLP [256, 256], 16
        # registers of width 16 with [256, 256] readouts; their weights
        # drawn like the rest (the network's own weights unchanged)
        m = copy.deepcopy(m)
        m.jas_mlp_width, m.jas_att_regs, m.jas_att_dim, m.jas_att_width = 256, 16, 16, 256
        pj = wl.init_params(s, m, np.random.default_rng(41))
        p = {k: (pj[k] if k.startswith(("jmlp_", "jatt_")) else v) for k, v in pj.items()}
        p.update({k: v for k, v in work.params[0].items()})
    F = fire.Fire(s, m, prec, max_walkers=W, cap_nbr=48, cap_upd=64, refresh_every=50, bf16_split=split)
    F.set_params(p)
    state, ws = F.buffers(W)
    R = torch.tensor(R0, dtype=torch.float64, device="cuda")
    Q = torch.tensor(wl.haar_rotations(W, np.random.default_rng(7)), device="cuda")
    n = s.n_el
    nsw = steps + warmup + 1
    xi, u = wl.noise_for(work, nsw, W)
    xi = torch.tensor(xi, device="cuda")
    u = torch.tensor(u, device="cuda")
    coeff = torch.full((W,), 1.0 / W, dtype=torch.float64, device="cuda")
    nacc = torch.zeros(W, dtype=torch.int32, device="cuda")
    # 10 burn-in proposals per electron are not timed: start from one sweep;
    # GEMM tile shapes are autotuned during the untimed burn-in and warm-up
    fire.autotune(True)
    F.eval_logpsi(R, state, ws)
    F.mcmc_sweep(R, state, ws, 1, work.step, xi[0:1].contiguous(), u[0:1].contiguous(), nacc)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ph = {"eval": 0.0, "sweep": 0.0, "local_energy": 0.0, "grad": 0.0}
    acc0 = None
    have_grad = want_grad
    last_e = None
    for it in range(warmup + steps):
        timed = it >= warmup
        if timed:
            fire.autotune(False)
        if timed and acc0 is None:
            acc0 = nacc.clone()
            if profile:
                F.profile_begin()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        ev[0].record(stream)
        F.eval_logpsi(R, state, ws)
        ev[1].record(stream)
        k = 1 + it
        F.mcmc_sweep(R, state, ws, 1, work.step, xi[k:k + 1].contiguous(), u[k:k + 1].contiguous(), nacc)
        ev[2].record(stream)
        e, parts, _, st = F.local_energy(R, state, ws, Q)
        ev[3].record(stream)
        if have_grad:
            try:
                F.grad_params(R, state, ws, coeff)
            except fire.FireError:
                have_grad = False
        ev[4].record(stream)
        torch.cuda.synchronize()
        print(f"# {prec} step {it} ({'timed' if timed else 'warmup'}): "
              f"{ev[0].elapsed_time(ev[4]):.0f} ms", file=sys.stderr, flush=True)
        if timed:
            ph["eval"] += ev[0].elapsed_time(ev[1])
            ph["sweep"] += ev[1].elapsed_time(ev[2])
            ph["local_energy"] += ev[2].elapsed_time(ev[3])
            ph["grad"] += ev[3].elapsed_time(ev[4])
            last_e = e
    prof = F.profile_end() if profile else None
    acc_rate = float((nacc - acc0).sum().item()) / (steps * W * n)
    # the local-energy phase again, serial and with stream overlap on (the
    # kinetic energy beside the pseudopotential, whose electrons alternate
    # between two streams), on the state the timed steps left; the other
    # phases do not change with it.  Not in the timed steps: overlapped
    # kernels share the chip, so their launch durations are not the
    # standalone rates the roofline needs.
    ovl = None
    if profile:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record(stream)
        e_s, _, _, _ = F.local_energy(R, state, ws, Q)
        ev[1].record(stream)
        F.set_overlap(True)
        F.local_energy(R, state, ws, Q)
        ev[2].record(stream)
        e_o, _, _, _ = F.local_energy(R, state, ws, Q)
        ev[3].record(stream)
        torch.cuda.synchronize()
        F.set_overlap(False)
        ovl = {"local_energy_ms_serial": ev[0].elapsed_time(ev[1]), "local_energy_ms": ev[2].elapsed_time(ev[3]),
               "max_abs_diff_vs_serial": float(torch.nan_to_num((e_o - e_s).abs(), 0.0).max().item())}
    # one sweep of global single-electron jumps (charge-weighted Gaussian
    # mixture over the nuclei, scale 2 bohr), after the timed steps
    gmm = None
    if profile:
        rg = np.random.default_rng(17)
        gxi = torch.tensor(rg.normal(size=(1, n, W, 3)), device="cuda")
        gu = torch.tensor(rg.uniform(size=(1, n, W)), device="cuda")
        gp = torch.tensor(wl.gmm_picks(1, n, W, rg), device="cuda")
        g0 = nacc.clone()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        _, _, _, gst = F.mcmc_sweep_mixed(R, state, ws, [1], work.step, 2.0, gxi, gu, gp, nacc)
        ev[1].record(stream)
        torch.cuda.synchronize()
        gmm = {"ms": ev[0].elapsed_time(ev[1]), "acceptance": float((nacc - g0).sum().item()) / (W * n),
               "walker_steps_per_s": W * n / (ev[0].elapsed_time(ev[1]) / 1e3),
               "flagged_walkers": int((gst != 0).sum().item())}
    # the S+ estimator for one spin-down electron: n_up two-electron swap
    # ratios per walker by low-rank updates, on the final state
    splus = None
    if profile:
        F.eval_logpsi(R, state, ws)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        _, rb, sst = F.splus_ratios(R, state, ws, s.n_up)
        ev[1].record(stream)
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1])
        splus = {"ms": t, "swap_ratios_per_s": W * s.n_up / (t / 1e3), "beta": s.n_up,
                 "flagged_walkers": int((sst != 0).sum().item()),
                 "mean_r_beta_squared": float(torch.nan_to_num(rb * rb).mean().item())}
    ph = {k: v / steps for k, v in ph.items()}
    if ovl is not None:
        # an estimate, not a measured step: the timed step with its
        # local-energy phase scaled by the overlapped / serial ratio of the
        # two calls above on the same state
        el = ph["local_energy"] * ovl["local_energy_ms"] / ovl["local_energy_ms_serial"]
        ovl["estimated_ms_per_step"] = sum(ph.values()) - ph["local_energy"] + el
        ovl["estimated_walkers_per_s"] = W / (ovl["estimated_ms_per_step"] / 1e3)
    e_np = last_e.cpu().numpy()
    out = dict(phases_ms=ph, ms_per_step=sum(ph.values()), acceptance=acc_rate, have_grad=have_grad,
               e_loc_mean=float(np.nanmean(e_np)), e_loc_median=float(np.nanmedian(e_np)),
               e_loc_nan=int(np.isnan(e_np).sum()))
    out["local_energies_per_s"] = W / (ph["local_energy"] / 1e3)
    out["walker_steps_per_s"] = W * n / (ph["sweep"] / 1e3)
    out["walkers_per_s"] = W / (out["ms_per_step"] / 1e3)
    out["prof"] = prof
    out["global_jump_sweep"] = gmm
    out["stream_overlap"] = ovl
    out["splus"] = splus
    if profile:
        out["counts"] = measured_counts(work, R.cpu().numpy(), work.step)
    return out


def measured_counts(work, R, step, sample=256, seed=5):
    """Neighbour and update-set counts on the walkers the timed steps left
    (a sample): |N_i| within c, |U| of a proposal of scale `step`, and
    pseudopotential (electron, atom) pairs within r_max per walker."""
    s, m = work.systems[0], work.model
    R = R[:sample]
    W, n = R.shape[:2]
    d = np.linalg.norm(R[:, :, None] - R[:, None], axis=-1)
    nb = (d <= m.cutoff).sum(-1) - 1
    rng = np.random.default_rng(seed)
    e = rng.integers(0, n, size=W)
    rn = R[np.arange(W), e] + step * rng.normal(size=(W, 3))
    d_old = d[np.arange(W), e]
    d_new = np.linalg.norm(R - rn[:, None], axis=-1)
    U = ((d_old <= m.cutoff) | (d_new <= m.cutoff)).sum(-1)
    dn = np.linalg.norm(R[:, :, None] - s.R_nuc[None, None], axis=-1)
    ecp = ((dn < s.ecp_rmax) & (s.species[None, None] == 1)).sum((1, 2)) if s.ecp else np.zeros(W)
    return {"walkers_sampled": int(W), "n_nb_mean": float(nb.mean()), "n_nb_max": int(nb.max()),
            "update_set_mean": float(U.mean()), "update_set_max": int(U.max()),
            "ecp_pairs_per_walker_mean": float(ecp.mean()), "ecp_pairs_per_walker_max": int(ecp.max())}


def run_tolerance(split, W=64):
    """The hybrid's stated E_L tolerance on a sample of the benchmark's
    walkers: E_L of the same W walkers in the BF16 hybrid and in FP64."""
    import torch
    import workloads as wl
    from paper_2504_06087_amd import fire

    work = wl.config(3, walkers=W)
    Q = torch.tensor(wl.haar_rotations(W, np.random.default_rng(7)), device="cuda")
    R = torch.tensor(work.R[0], dtype=torch.float64, device="cuda")
    e = {}
    for prec, sp in (("fp64", 0), ("bf16", split)):
        F = fire.Fire(work.systems[0], work.model, prec, max_walkers=W, cap_nbr=48, cap_upd=64, bf16_split=sp)
        F.set_params(work.params[0])
        state, ws = F.buffers(W)
        F.eval_logpsi(R, state, ws)
        e[prec], _, _, _ = F.local_energy(R, state, ws, Q)
        torch.cuda.synchronize()
        e[prec] = e[prec].cpu().numpy()
        del F, state, ws
        torch.cuda.empty_cache()
    d = e["bf16"] - e["fp64"]

    def clipped(x):
        # the paper's local-energy clipping for the gradient: 5 mean
        # absolute deviations around the median
        med = np.median(x)
        mae = np.mean(np.abs(x - med))
        return np.clip(x, med - 5 * mae, med + 5 * mae)
    dc = clipped(e["bf16"]) - clipped(e["fp64"])
    return {"walkers": W, "bar_ha": 1e-3, "batch_mean_diff_ha": float(np.mean(d)),
            "median_abs_diff_ha": float(np.median(np.abs(d))), "max_abs_diff_ha": float(np.abs(d).max()),
            "clipped_batch_mean_diff_ha": float(np.mean(dc)), "met": bool(abs(np.mean(d)) <= 1e-3)}


def run_spring(W=256):
    """One natural-gradient step at the benchmark's molecule and network:
    the per-walker gradients [W][P] (the adjoint one walker at a time), then
    the W x W Gram matrix, its centring and the FP64 Cholesky solve."""
    import torch
    import workloads as wl
    from paper_2504_06087_amd import fire

    work = wl.config(3, walkers=W)
    F = fire.Fire(work.systems[0], work.model, "bf16", max_walkers=W, cap_nbr=48, cap_upd=64, bf16_split=7)
    F.set_params(work.params[0])
    state, ws = F.buffers(W)
    R = torch.tensor(work.R[0], dtype=torch.float64, device="cuda")
    Q = torch.tensor(wl.haar_rotations(W, np.random.default_rng(7)), device="cuda")
    O = torch.empty(W, F.P, dtype=torch.float64, device="cuda")
    F.eval_logpsi(R, state, ws)
    e, _, _, _ = F.local_energy(R, state, ws, Q)
    coeff = torch.zeros(W, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record(stream)
    F.grad_params(R, state, ws, coeff, per_walker=O)
    ev[1].record(stream)
    delta, info = F.spring_step(O, e, ws, 1e-3, 0.99)
    ev[2].record(stream)
    torch.cuda.synchronize()
    return {"walkers": W, "parameters": F.P, "per_walker_grad_ms": ev[0].elapsed_time(ev[1]),
            "spring_step_ms": ev[1].elapsed_time(ev[2]), "info": int(info.item()),
            "delta_norm": float(delta.norm().item())}


def run_el_rule(split, W, n_quad):
    """The local-energy phase of the same workload with an n_quad-point
    pseudopotential rule on C instead of the 12-point one (the paper's
    per-species choice is 4 points for Li-Ne): one untimed and one timed
    call after a full evaluation."""
    import copy
    import torch
    import workloads as wl
    from paper_2504_06087_amd import fire

    work = wl.config(3, walkers=W)
    s = copy.deepcopy(work.systems[0])
    s.ecp_nquad = {1: n_quad}
    F = fire.Fire(s, work.model, "bf16", max_walkers=W, cap_nbr=48, cap_upd=64, refresh_every=50,
                  bf16_split=split)
    F.set_params(work.params[0])
    state, ws = F.buffers(W)
    R = torch.tensor(work.R[0], dtype=torch.float64, device="cuda")
    Q = torch.tensor(wl.haar_rotations(W, np.random.default_rng(7)), device="cuda")
    F.eval_logpsi(R, state, ws)
    stream = torch.cuda.current_stream()
    ms = []
    for _ in range(2):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record(stream)
        F.local_energy(R, state, ws, Q)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    return {"n_quad_on_C": n_quad, "local_energy_ms": ms[-1], "local_energies_per_s_el_phase": W / (ms[-1] / 1e3)}


def run_c5(split, W, steps, warmup):
    """The uneven batch: 16 systems (H chains and C/H flakes, 20-180 valence
    electrons) x W walkers, shared embedding, per-system orbitals; one step =
    evaluation + 1 sweep + local energy + energy gradient for every system,
    replayed as one captured graph after an autotuning step."""
    import torch
    import workloads as wl
    from paper_2504_06087_amd import fire

    work = wl.config(4, walkers=W)
    shared, private = wl.batch_params(work.params)
    nsys = len(work.systems)
    B = fire.FireBatch(work.systems, work.model, "bf16", [W] * nsys, cap_nbr=48, cap_upd=64, bf16_split=split)
    B.set_params(B.flatten(shared, private))
    R = B.concat(work.R)
    nsw = steps + warmup + 2
    per = [wl.noise_for(work, nsw, W, system=k) for k in range(nsys)]
    xi_all = [B.concat([per[k][0][t:t + 1] for k in range(nsys)]) for t in range(nsw)]
    u_all = [B.concat([per[k][1][t:t + 1] for k in range(nsys)]) for t in range(nsw)]
    xi, u = xi_all[0].clone(), u_all[0].clone()
    state, ws = B.buffers(1)
    nacc = torch.zeros(nsys * W, dtype=torch.int32, device="cuda")
    out = B.outputs()
    stream = torch.cuda.current_stream()
    # eager step with the tile autotuner on
    fire.autotune_clear()
    fire.autotune(True)
    t0 = time.time()
    B.step(R, state, ws, 1, work.step, xi, u, nacc, out=out)
    torch.cuda.synchronize()
    t_tune = time.time() - t0
    fire.autotune(False)
    tuned = fire.autotune_count()
    # eager step (tuned tiles)
    xi.copy_(xi_all[1])
    u.copy_(u_all[1])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    B.step(R, state, ws, 1, work.step, xi, u, nacc, out=out)
    ev[1].record(stream)
    torch.cuda.synchronize()
    eager_ms = ev[0].elapsed_time(ev[1])
    print(f"# c5 eager step: {eager_ms:.0f} ms (tuning step {t_tune:.1f} s, {tuned} shapes)", file=sys.stderr,
          flush=True)
    t0 = time.time()
    G = B.graph(R, state, ws, 1, work.step, xi, u, nacc, out)
    t_cap = time.time() - t0
    ms = 0.0
    acc0 = None
    for it in range(warmup + steps):
        xi.copy_(xi_all[2 + it])
        u.copy_(u_all[2 + it])
        if it == warmup:
            acc0 = nacc.clone()
        torch.cuda.synchronize()
        ev[0].record(stream)
        G.launch()
        ev[1].record(stream)
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1])
        print(f"# c5 graph step {it} ({'timed' if it >= warmup else 'warmup'}): {t:.0f} ms", file=sys.stderr,
              flush=True)
        if it >= warmup:
            ms += t
    ms /= steps
    e = out[0]
    n_el = [s.n_el for s in work.systems]
    tot_w = nsys * W
    acc = float((nacc - acc0).sum().item()) / (steps * W * sum(n_el))
    return {
        "workload": f"16 systems (H chains and C/H flakes), valence electrons {sorted(n_el)}, {W} walkers each, "
                    f"width 256, 3 layers, 4 determinants, c = 5 bohr, local pseudopotential on C; step = "
                    f"evaluation + 1 sweep + local energy + energy gradient per system, one graph launch",
        "ms_per_step": ms, "eager_ms_per_step": eager_ms, "walkers_per_s": tot_w / (ms / 1e3),
        "walker_steps_per_s_incl_step": W * sum(n_el) / (ms / 1e3), "acceptance": acc,
        "tuned_gemm_shapes": tuned, "capture_s": t_cap,
        "e_loc_nan": int(torch.isnan(e).sum().item()),
    }


def fit_exponent(n, t):
    """eta of the least-squares power law t ~ n**eta (a line in log-log)."""
    x, y = np.log(np.asarray(n, float)), np.log(np.asarray(t, float))
    return float(np.polyfit(x, y, 1)[0])


def paper_step_model(t_wf, t_upd, t_kin, n, n_sweeps=2, n_quad=4):
    """Total time of one optimisation step composed from the measured update,
    evaluation and kinetic times as in the paper's runtime study (Appendix,
    runtime comparison): sampling T_wf + N_sweeps n T_upd, the pseudopotential
    n N_quad T_upd and the spin operator n/2 T_upd, plus T_kin."""
    return t_wf + n_sweeps * n * t_upd + t_kin + n * n_quad * t_upd + 0.5 * n * t_upd


def run_scaling(carbons, W, split, cutoff):
    """Runtime scaling on cumulenes H2C=(C=)kCH2 (Fig. 2a-c of the paper):
    per chain length, the times of a full evaluation (T_wf), of one
    single-electron update over all walkers (T_upd = sweep / n), of the
    local energy without the nonlocal pseudopotential (T_kin = E_L call minus
    the V_NL call), of the V_NL call, and of the gradient; fitted exponents
    eta of T ~ n**eta."""
    import torch
    import workloads as wl
    from paper_2504_06087_amd import fire

    pts = []
    for nc in carbons:
        rng = np.random.default_rng(wl.BASE_SEED + 1000 + nc)
        Rn, sp = wl.cumulene(nc)
        s = wl.make_system(f"C{nc}H4", Rn, sp, pseudo_c=True, nonlocal_ecp=True, ecp_rng=rng, per_species=True)
        m = wl.make_model(s, width=256, mlp_layers=3, n_det=16, n_env=8, cutoff=cutoff, cutoff_nuc=20.0)
        p = wl.init_params(s, m, rng)
        n = s.n_el
        F = fire.Fire(s, m, "bf16", max_walkers=W, cap_nbr=48, cap_upd=64, refresh_every=50, bf16_split=split)
        F.set_params(p)
        state, ws = F.buffers(W)
        R = torch.tensor(wl.init_walkers(s, W, rng), dtype=torch.float64, device="cuda")
        Q = torch.tensor(wl.haar_rotations(W, rng), device="cuda")
        xi, u = wl.mcmc_noise(3, n, W, rng)
        xi, u = torch.tensor(xi, device="cuda"), torch.tensor(u, device="cuda")
        coeff = torch.full((W,), 1.0 / W, dtype=torch.float64, device="cuda")
        nacc = torch.zeros(W, dtype=torch.int32, device="cuda")
        stream = torch.cuda.current_stream()
        times = None
        # pass 0: burn-in with the tile autotuner on; pass 1 timed
        for it in range(2):
            fire.autotune(it == 0)
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
            ev[0].record(stream)
            F.eval_logpsi(R, state, ws)
            ev[1].record(stream)
            F.mcmc_sweep(R, state, ws, 1, 0.2, xi[it:it + 1].contiguous(), u[it:it + 1].contiguous(), nacc)
            ev[2].record(stream)
            F.ecp_nonlocal(R, state, ws, Q)
            ev[3].record(stream)
            F.local_energy(R, state, ws, Q)
            ev[4].record(stream)
            F.grad_params(R, state, ws, coeff)
            ev[5].record(stream)
            torch.cuda.synchronize()
            times = [ev[k].elapsed_time(ev[k + 1]) for k in range(5)]
            print(f"# cumulene C{nc}H4 n={n} pass {it}: " + " ".join(f"{t:.1f}" for t in times) + " ms",
                  file=sys.stderr, flush=True)
        t_wf, t_sw, t_ecp, t_el, t_gr = times
        t_upd = t_sw / n
        t_kin = t_el - t_ecp
        pts.append({"n_carbon": nc, "n_el": n, "t_wf_ms": t_wf, "t_upd_ms": t_upd, "t_sweep_ms": t_sw,
                    "t_kin_ms": t_kin, "t_vnl_ms": t_ecp, "t_el_ms": t_el, "t_grad_ms": t_gr,
                    "t_tot_model_ms": paper_step_model(t_wf, t_upd, t_kin, n),
                    "t_step_measured_ms": t_wf + t_sw + t_el + t_gr})
        del F, state, ws
        torch.cuda.empty_cache()
    fire.autotune(False)
    ns = [q["n_el"] for q in pts]
    fits = {}
    for key in ("t_upd_ms", "t_kin_ms", "t_wf_ms", "t_tot_model_ms", "t_step_measured_ms"):
        ts = [q[key] for q in pts]
        fits[key] = {"all": fit_exponent(ns, ts)}
        big = [(a, b) for a, b in zip(ns, ts) if a >= 100]
        if len(big) >= 2:
            fits[key]["n_el>=100"] = fit_exponent([a for a, _ in big], [b for _, b in big])
    return {"metric": "cumulene runtime scaling (T ~ n_el^eta)", "walkers": W, "cutoff_bohr": cutoff,
            "model": "width 256, 3 layers, 16 determinants, 8 envelopes, BF16-hybrid",
            "points": pts, "eta": fits}


def cpu_baseline():
    """The FP64 oracle on the host cores, on a bounded sample of the same
    workload: one walker's forward pass, gradient, 12 of the 540 Hessian
    diagonal entries and 24 pseudopotential ratios, scaled per walker."""
    import torch
    import workloads as wl
    from oracle import Oracle

    torch.set_num_threads(os.cpu_count() or 1)
    work = wl.config(3, walkers=1)
    s, m, p, R = work.systems[0], work.model, work.params[0], work.R[0]
    O = Oracle(s, m, p)
    t0 = time.time()
    O.log_psi(R)
    t_fwd = time.time() - t0
    coords = np.arange(0, 3 * s.n_el, 45)[:12]
    t0 = time.time()
    O.grad_lap(R, chunk=12, coords=coords)
    t_lap = time.time() - t0
    # pseudopotential ratios of this walker: count pairs, time 24 full recomputes
    d = np.linalg.norm(R[0][:, None, :] - s.R_nuc[None], axis=-1)
    pairs = int(((d < s.ecp_rmax) & (s.species[None] == 1)).sum())
    Rq = np.repeat(R, 24, axis=0)
    t0 = time.time()
    O.log_psi(Rq)
    t_24 = time.time() - t0
    t_el = t_fwd + t_lap * (3 * s.n_el / len(coords)) + t_24 * (12 * pairs / 24.0)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": 1.0 / t_el, "unit": "local energies/s", "cores": torch.get_num_threads(), "kind": "oracle",
        "cpu_model": model,
        "walker_steps_per_s": 1.0 / t_fwd,
        "sample": (f"1 walker of the same workload: forward ({t_fwd:.2f}s), gradient + 12 of {3 * s.n_el} Hessian "
                   f"diagonal entries ({t_lap:.2f}s, scaled x{3 * s.n_el / len(coords):.0f}), 24 of {12 * pairs} "
                   f"quadrature ratios ({t_24:.2f}s, scaled); a Metropolis walker-step is one full forward"),
    }


def model_roofline(hyb):
    """Whole-phase fractions of the cost model's ceilings: local energies
    against the ~100 GFLOP per walker of the model at the BF16 peak, and
    walker-steps against the bytes a proposal moves with the measured update
    set and acceptance (FP64 inverse)."""
    c = hyb.get("counts") or {}
    U = c.get("update_set_mean", 26.3)
    acc = hyb.get("acceptance", 0.5)
    n, d, K, N = 180, 256, 16, 90
    bytes_step = 24 * n + 10 * U * d + 4 * U * K * N + 8 * N * U * K + acc * 4 * K * N * N * 8
    el = hyb["local_energies_per_s"]
    ws = hyb["walker_steps_per_s"]
    return {"e_loc_gflop_per_walker": 100.0, "e_loc_frac_of_bf16_peak": el * 100e9 / 2.5e15,
            "walker_step_bytes": bytes_step, "walker_step_frac_of_hbm": ws * bytes_step / HBM_PEAK}


def main():
    a = parse()
    if a.copy_probe:
        copy_probe()
        return
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (walkers shard across GPUs "
                                   "without communication inside a step, see the design notes)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    W = a.walkers
    if a.scaling:
        res = run_scaling([int(x) for x in a.scaling_carbons.split(",")], W, a.split, a.scaling_cutoff)
        print(json.dumps(res), flush=True)
        return
    hyb = run_precision("bf16", a.split, W, a.steps, a.warmup, not a.no_grad, profile=True)
    print(f"# hybrid: {json.dumps({k: v for k, v in hyb.items() if k != 'prof'})}", flush=True)
    print(f"# hybrid GEMM profile: {hyb['prof']}", flush=True)
    jas = None
    if a.jastrow:
        torch.cuda.empty_cache()
        jas = run_precision("bf16", a.split, W, a.steps, a.warmup, not a.no_grad, profile=False, jastrow=True)
        jas = {k: v for k, v in jas.items() if k not in ("prof", "counts")}
        print(f"# hybrid with the MLP and attention Jastrows: {json.dumps(jas)}", flush=True)
    rule4 = None
    if not a.no_rule4:
        torch.cuda.empty_cache()
        rule4 = run_el_rule(a.split, W, 4)
        print(f"# E_L with the 4-point rule on C: {json.dumps(rule4)}", flush=True)
    fp32 = None
    if not a.no_fp32:
        torch.cuda.empty_cache()
        fp32 = run_precision("fp32", 0, W, a.steps, a.warmup, not a.no_grad, profile=False)
        print(f"# fp32: {json.dumps({k: v for k, v in fp32.items() if k != 'prof'})}", flush=True)
    # roofline of the dominant kernel: the MFMA GEMM of the hybrid path.
    # Algorithmic flops and bytes come from each launch's actual row count;
    # the bound is HBM when the flops per byte fall below the ridge point.
    prof = hyb["prof"] or {}
    kind = max(prof, key=lambda k: prof[k][1]) if prof else "bf16x3"
    la, ms, fl, by = prof.get(kind, (0, 0.0, 0.0, 0.0))
    sec = ms / 1e3
    tflops = fl / sec / 1e12 if sec > 0 else 0.0
    gbs = by / sec / 1e9 if sec > 0 else 0.0
    hbm_bound = by > 0 and fl / by < PEAK[kind] / HBM_PEAK
    traffic = measured_traffic() if kind == "bf16x3" else None
    roof = {"bound": "hbm" if hbm_bound else "mfma", "kernel": f"k_gemm<{kind}>",
            "achieved": gbs if hbm_bound else tflops, "peak": HBM_PEAK / 1e9 if hbm_bound else PEAK[kind] / 1e12,
            "unit": "GB/s" if hbm_bound else "TFLOP/s",
            "frac": (gbs * 1e9 / HBM_PEAK) if hbm_bound else (tflops * 1e12 / PEAK[kind]),
            "traffic": traffic,
            "launches": la, "kernel_ms_per_step": ms / a.steps, "mean_launch_us": 1e3 * ms / max(1, la),
            "algorithmic_bytes_per_launch": by / max(1, la), "flops_per_launch": fl / max(1, la),
            "achieved_tflops": tflops, "mfma_frac": tflops * 1e12 / PEAK[kind],
            "achieved_gbs": gbs, "hbm_frac": gbs * 1e9 / HBM_PEAK}
    c5 = None
    if not a.no_c5:
        torch.cuda.empty_cache()
        c5 = run_c5(a.split, a.c5_walkers, a.steps, a.warmup)
        print(f"# c5: {json.dumps(c5)}", flush=True)
    torch.cuda.empty_cache()
    tol = run_tolerance(a.split)
    print(f"# hybrid E_L tolerance: {json.dumps(tol)}", flush=True)
    torch.cuda.empty_cache()
    spring = run_spring()
    print(f"# spring: {json.dumps(spring)}", flush=True)
    cpu = None if a.no_cpu else cpu_baseline()
    line = {
        "metric": METRIC, "value": hyb["walkers_per_s"], "unit": "local energies/s", "n_gpus": 1,
        "steps": a.steps, "warmup": a.warmup, "ms_per_step": hyb["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16", "data": "synthetic",
        "config": {"workload": f"C42H12 flake, 180 valence electrons (90 up, 90 down), {W} walkers, width 256, "
                               "3 MLP layers, 16 determinants, c = 5 bohr, c_n = 20 bohr, nonlocal l = 0,1 "
                               "pseudopotential on C with a 12-point rule; step = full evaluation + 1 Metropolis "
                               "sweep + local energy + parameter gradient",
                   "walkers": W, "electrons": 180, "precision": f"bf16 hybrid (split sites {a.split}), FP64 LU"},
        "walker_steps_per_s": hyb["walker_steps_per_s"],
        "local_energies_per_s_el_phase": hyb["local_energies_per_s"],
        "phases_ms": hyb["phases_ms"], "acceptance": hyb["acceptance"], "grad_included": hyb["have_grad"],
        "global_jump_sweep": hyb.get("global_jump_sweep"),
        "stream_overlap": hyb.get("stream_overlap"),
        "local_energy_4point_rule": rule4,
        "step_with_neural_jastrows": jas,
        "hybrid_e_loc_tolerance": tol,
        "measured_counts": hyb.get("counts"),
        "model_roofline": model_roofline(hyb),
        "splus_estimator": hyb.get("splus"),
        "spring_step": spring,
        "fp32_plain": None if fp32 is None else {
            "value": fp32["walkers_per_s"], "ms_per_step": fp32["ms_per_step"], "phases_ms": fp32["phases_ms"],
            "walker_steps_per_s": fp32["walker_steps_per_s"],
            "local_energies_per_s_el_phase": fp32["local_energies_per_s"]},
        "roofline": roof,
        "uneven_batch": c5,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
