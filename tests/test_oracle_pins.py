"""Pins of the FP64 oracle against what the paper and mathematics fix.

Each test names the passage it follows.  None of them re-types an oracle
formula: they check closed forms in special parameter settings, exact
symmetries, limits, textbook routines and finite differences.
"""
import copy
import math

import numpy as np
import pytest
import torch

import workloads as wl
from oracle import Oracle, fcut, silu

DT = torch.float64


def _orc(cid=0, W=4, **model_kw):
    w = wl.config(cid, walkers=W)
    s, m, p = w.systems[0], copy.deepcopy(w.model), copy.deepcopy(w.params[0])
    for k, v in model_kw.items():
        setattr(m, k, v)
    return s, m, p, w.R[0]


def _small_c2(W=2, n_keep=None):
    """Polyene with a narrow network so that CPU autodiff stays fast."""
    R, sp = wl.polyene_c12h14()
    s = wl.make_system("C12H14", R, sp, pseudo_c=True)
    m = wl.make_model(s, width=16, mlp_layers=2, n_det=2, n_env=2, cutoff=5.0, cutoff_nuc=20.0)
    rng = np.random.default_rng(7)
    p = wl.init_params(s, m, rng)
    return s, m, p, wl.init_walkers(s, W, rng)


# --------------------------------------------------------------------------
# cutoff function (Methods, spatial filters: smooth decay to 0 at the cutoff)
# --------------------------------------------------------------------------
def test_fcut_endpoints_and_smoothness():
    x = torch.tensor([0.0, 1.0, 1.3, 7.0])
    v = fcut(x)
    assert v[0] == 1.0 and v[1] == 0.0 and v[2] == 0.0 and v[3] == 0.0
    h = 1e-4
    xs = torch.tensor([1.0 - 2 * h, 1.0 - h, 1.0])
    f = fcut(xs)
    # one-sided first and second differences at x = 1 vanish as O(h^2) and
    # O(h): the function is C2 across the cutoff (leading term 56 (1-x)^3)
    assert abs((f[2] - f[1]) / h) < 100 * h * h
    assert abs((f[2] - 2 * f[1] + f[0]) / h ** 2) < 1000 * h
    assert abs(float(f[1]) / h ** 3 - 56.0) < 0.1
    # monotone decreasing on [0, 1]
    g = fcut(torch.linspace(0, 1, 200))
    assert torch.all(g[1:] <= g[:-1] + 1e-15)


# --------------------------------------------------------------------------
# hydrogen: exact ground state (Methods, Hamiltonian and local energy)
# --------------------------------------------------------------------------
def test_hydrogen_local_energy_is_minus_half():
    s, m, p, R = wl.hydrogen_atom(W=12, seed=3)
    o = Oracle(s, m, p)
    e, parts = o.local_energy(R)
    assert torch.allclose(e, torch.full_like(e, -0.5), atol=1e-10, rtol=0)
    # kinetic = 1/r - 1/2 and V_en = -1/r separately
    r = np.linalg.norm(R[:, 0], axis=1)
    assert np.allclose(parts[:, 0].numpy(), 1.0 / r - 0.5, atol=1e-10)
    assert np.allclose(parts[:, 2].numpy(), -1.0 / r, atol=1e-12)


def test_zero_variance_energy_gradient_vanishes():
    from oracle import energy_gradient
    s, m, p, R = wl.hydrogen_atom(W=8, seed=4)
    o = Oracle(s, m, p)
    e, _ = o.local_energy(R)
    g = energy_gradient(o, R, e)
    assert max(float(v.abs().max()) for v in g.values() if v.numel()) < 1e-11


def test_hydrogen_sampling_mean_radius():
    """|psi|^2 = exp(-2r)/pi: <r> = 3/2 bohr (textbook 1s value)."""
    s, m, p, R = wl.hydrogen_atom(W=512, seed=5)
    o = Oracle(s, m, p)
    rng = np.random.default_rng(11)
    R = R * 0.5
    rs = []
    for blk in range(30):
        xi, u = wl.mcmc_noise(10, 1, 512, rng)
        R, _, _, _ = o.mcmc_sweep(R, 1.0, xi, u)
        if blk >= 8:
            rs.append(np.linalg.norm(R.numpy()[:, 0], axis=1).mean())
    assert abs(np.mean(rs) - 1.5) < 0.03


# --------------------------------------------------------------------------
# symmetries (Introduction: antisymmetry from determinants; features are
# differences of positions)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("which", ["h4", "c2"])
def test_antisymmetry_same_spin_swap(which):
    if which == "h4":
        s, m, p, R = _orc(0, W=3)
        pairs = [(0, 1), (2, 3)]
    else:
        s, m, p, R = _small_c2(W=2)
        pairs = [(0, 5), (31, 40)]
    o = Oracle(s, m, p)
    s0, l0 = o.log_psi(R)
    for i, j in pairs:
        R2 = R.copy()
        R2[:, [i, j]] = R2[:, [j, i]]
        s1, l1 = o.log_psi(R2)
        assert torch.all(s1 == -s0)
        assert torch.allclose(l1, l0, atol=1e-12, rtol=0)


def test_opposite_spin_swap_is_not_a_symmetry():
    s, m, p, R = _orc(0, W=3)
    o = Oracle(s, m, p)
    _, l0 = o.log_psi(R)
    R2 = R.copy()
    R2[:, [0, 2]] = R2[:, [2, 0]]
    _, l1 = o.log_psi(R2)
    assert (l1 - l0).abs().max() > 1e-3


def test_translation_invariance():
    s, m, p, R = _small_c2(W=2)
    o = Oracle(s, m, p)
    _, l0 = o.log_psi(R)
    shift = np.array([0.37, -1.21, 0.55])
    s2 = copy.deepcopy(s)
    s2.R_nuc = s.R_nuc + shift
    o2 = Oracle(s2, m, p)
    _, l1 = o2.log_psi(R + shift)
    assert torch.allclose(l0, l1, atol=1e-9, rtol=1e-12)


def test_same_spin_permutation_equivariance_of_embeddings():
    s, m, p, R = _small_c2(W=1)
    o = Oracle(s, m, p)
    perm = np.arange(s.n_el)
    perm[[3, 17]] = perm[[17, 3]]
    h = o.embed(torch.tensor(R))["h"]
    hp = o.embed(torch.tensor(R[:, perm]))["h"]
    assert torch.allclose(hp, h[:, perm], atol=1e-12, rtol=0)


# --------------------------------------------------------------------------
# locality (Introduction, finite-range neighbourhood N_i)
# --------------------------------------------------------------------------
def test_embedding_locality_and_dependence_within_cutoff():
    s, m, p, R = _small_c2(W=1)
    o = Oracle(s, m, p)
    R = R.copy()
    i, j = 0, 20
    ri = R[0, i]
    # place j farther than c from r_i, then move it to another far point
    R[0, j] = ri + np.array([6.0, 0.0, 0.0])
    h_a = o.embed(torch.tensor(R))["h"][0, i].clone()
    R2 = R.copy()
    R2[0, j] = ri + np.array([0.0, -7.5, 1.0])
    h_b = o.embed(torch.tensor(R2))["h"][0, i]
    assert torch.equal(h_a, h_b)
    # within the cutoff the embedding does depend on r_j
    R3 = R.copy()
    R3[0, j] = ri + np.array([1.5, 0.3, 0.0])
    h_c = o.embed(torch.tensor(R3))["h"][0, i]
    assert (h_c - h_a).abs().max() > 1e-6


# --------------------------------------------------------------------------
# closed forms under special parameter choices
# --------------------------------------------------------------------------
def _shift(d, k=1):
    P = np.zeros((d, d))
    for c in range(d):
        P[c, (c + k) % d] = 1.0     # (x P)[c+k] = x[c]
    return P


def test_message_closed_form():
    """Filters reduced to SiLU(1) * f_cut(r/c) exp(-sigma_1^2 r^2) and the
    message MLP to SiLU(h0_i[c-1] + x-direction feature + beta_alpha):
    m^alpha_i[c] = sum over same/opposite spin j != i, |r_ij| <= c."""
    s, m, p, R = _small_c2(W=1)
    d = m.width
    for a in (0, 1):
        p["ee_W1"][a][:] = 0.0
        p["ee_b1"][a][:] = 0.0
        p["ee_W2"][a][:] = 0.0
        p["ee_b2"][a][:] = 1.0
        p["ee_W3"][a][:] = 1.0 / m.edge_hidden[1]
        p["ee_Wenv"][a][:] = 0.0
        p["ee_Wenv"][a][0, :] = 1.0
        p["msg_Wa"][a] = _shift(d) if a == 0 else np.zeros((d, d))
        p["msg_Wb"][a] = np.zeros((d, d)) if a == 0 else _shift(d, 2)
        p["msg_We"][a][:] = 0.0
        p["msg_We"][a][1, :] = 1.0
        p["msg_b"][a][:] = 0.3 + a
    o = Oracle(s, m, p)
    out = o.embed(torch.tensor(R))
    h0 = out["h0"][0].numpy()
    n, nu = s.n_el, s.n_up
    pos = R[0]
    sig = p["ee_sig"][:, 0]
    for a in (0, 1):
        got = out["m"][a][0].numpy()
        exp = np.zeros((n, d))
        for i in range(n):
            for j in range(n):
                same = (i < nu) == (j < nu)
                if i == j or same != (a == 0):
                    continue
                dv = pos[i] - pos[j]
                r = np.linalg.norm(dv)
                if r >= m.cutoff:
                    continue
                x = r / m.cutoff
                u = 1 - 28 * x ** 6 + 48 * x ** 7 - 21 * x ** 8
                gam = (1 / (1 + np.exp(-1.0))) * 1.0 * u * np.exp(-sig[a] ** 2 * r * r)
                src = np.roll(h0[i], 1) if a == 0 else np.roll(h0[j], 2)
                pre = src + math.log1p(r) / r * dv[0] + (0.3 + a)
                exp[i] += gam * pre / (1 + np.exp(-pre))
        assert np.allclose(got, exp, atol=1e-12, rtol=1e-12)


def test_electron_nucleus_embedding_closed_form():
    """Gamma_m reduced to SiLU(SiLU(b1_m)) f_cut(rho/c_n) exp(-sigma_1^2 rho^2)
    with a per-nucleus bias; value part nuc_emb_m + log(1+rho)/rho * (x_i -
    X_m)_y."""
    s, m, p, R = _small_c2(W=1)
    d = m.width
    M = s.n_nuc
    rng = np.random.default_rng(2)
    p["en_W1"][:] = 0.0
    p["en_b1"][:] = 0.0
    p["en_b1"][:, 0] = rng.normal(size=M)
    p["en_W2"][:] = 0.0
    p["en_W2"][0, :] = 1.0
    p["en_b2"][:] = 0.0
    p["en_W3"][:] = 1.0 / m.edge_hidden[1]
    p["en_Wenv"][:] = 0.0
    p["en_Wenv"][0, :] = 1.0
    p["en_Wn"][:] = 0.0
    p["en_Wn"][2, :] = 1.0
    o = Oracle(s, m, p)
    got = o.embed(torch.tensor(R))["s"][0].numpy()
    sl = lambda x: x / (1 + np.exp(-x))
    exp = np.zeros((s.n_el, d))
    for i in range(s.n_el):
        for mm in range(M):
            dv = R[0, i] - s.R_nuc[mm]
            rho = np.linalg.norm(dv)
            if rho >= m.cutoff_nuc:
                continue
            x = rho / m.cutoff_nuc
            u = 1 - 28 * x ** 6 + 48 * x ** 7 - 21 * x ** 8
            g = sl(sl(p["en_b1"][mm, 0])) * u * np.exp(-p["en_sig"][0] ** 2 * rho ** 2)
            exp[i] += g * (p["nuc_emb"][mm] + math.log1p(rho) / rho * dv[1])
    assert np.allclose(got, exp, atol=1e-11, rtol=1e-12)


def test_layernorm_and_glu_orientation():
    """LN over channels (mean beta, biased variance gamma^2 var/(var+eps));
    GLU with W_v a cyclic shift, gate constant: h0 = SiLU(b_g) * LN(s) shifted."""
    s, m, p, R = _small_c2(W=1)
    d = m.width
    p["glu_Wv"] = _shift(d, 3)
    p["glu_bv"][:] = 0.0
    p["glu_Wg"][:] = 0.0
    p["glu_bg"][:] = 2.5
    p["glu_Wo"] = np.eye(d)
    p["glu_bo"][:] = 0.0
    o = Oracle(s, m, p)
    out = o.embed(torch.tensor(R))
    sv = out["s"][0].numpy()
    mu = sv.mean(1, keepdims=True)
    var = sv.var(1, keepdims=True)
    ln = (sv - mu) / np.sqrt(var + 1e-5)
    assert np.allclose(ln.mean(1), 0.0, atol=1e-12)
    exp = np.roll(ln, 3, axis=1) * (2.5 / (1 + math.exp(-2.5)))
    assert np.allclose(out["h0"][0].numpy(), exp, atol=1e-12)


def test_mlp_orientation():
    s, m, p, R = _small_c2(W=1)
    d = m.width
    p["mlp_W"][0] = _shift(d, 1)
    p["mlp_b"][0][:] = 0.1
    p["mlp_W"][1] = np.eye(d)
    p["mlp_b"][1][:] = 0.0
    o = Oracle(s, m, p)
    out = o.embed(torch.tensor(R))
    h1 = out["h1"][0].numpy()
    sl = lambda x: x / (1 + np.exp(-x))
    exp = sl(sl(np.roll(h1, 1, axis=1) + 0.1))
    assert np.allclose(out["h"][0].numpy(), exp, atol=1e-12)


# --------------------------------------------------------------------------
# c = 0 limit (Introduction: c = 0 gives single-electron orbitals): textbook
# Slater-determinant kinetic energy
# --------------------------------------------------------------------------
def test_zero_cutoff_slater_kinetic_textbook():
    s, m, p, R = _orc(0, W=2)
    m.cutoff = 1e-9
    o = Oracle(s, m, p)
    R = R.copy()
    kin = o.kinetic(R).numpy()
    _, lap = o.grad_lap(R)
    nu, n = s.n_up, s.n_el
    h = 2e-3

    def orb_rows(Rw, i):
        """Row i of the spin block of electron i, all dets: [K, N]."""
        out = o.embed(torch.tensor(Rw[None]))["h"]
        phis = o.orbitals(torch.tensor(Rw[None]), out)
        blk = 0 if i < nu else 1
        row = i if i < nu else i - nu
        return phis[blk][0, :, row, :].numpy()

    for w in range(R.shape[0]):
        tot = 0.0
        phis = o.orbitals(torch.tensor(R[w:w + 1]), o.embed(torch.tensor(R[w:w + 1]))["h"])
        inv = [np.linalg.inv(ph[0, 0].numpy()) for ph in phis]
        for i in range(n):
            blk = 0 if i < nu else 1
            row = i if i < nu else i - nu
            lapl = np.zeros(inv[blk].shape[0])
            f0 = orb_rows(R[w], i)[0]
            for x in range(3):
                acc = -30 * f0
                for k, c in ((1, 16), (2, -1)):
                    for sgn in (1, -1):
                        Rp = R[w].copy()
                        Rp[i, x] += sgn * k * h
                        acc = acc + c * orb_rows(Rp, i)[0]
                lapl += acc / (12 * h * h)
            tot += lapl @ inv[blk][:, row]
        assert abs(-0.5 * tot - kin[w]) < 1e-6 * max(1.0, abs(kin[w]))


# --------------------------------------------------------------------------
# derivatives against central finite differences (Methods, local energy)
# --------------------------------------------------------------------------
def test_gradient_and_laplacian_vs_finite_differences():
    s, m, p, R = _orc(0, W=2)
    o = Oracle(s, m, p)
    g, lap = o.grad_lap(R)
    h = 1e-3
    for w in range(2):
        x0 = R[w].copy()
        f = lambda x: float(o.log_psi(x[None])[1][0])
        l0 = f(x0)
        fd_lap, fd_g = 0.0, np.zeros_like(x0)
        for i in range(s.n_el):
            for k in range(3):
                vals = {}
                for st in (-2, -1, 1, 2):
                    x = x0.copy()
                    x[i, k] += st * h
                    vals[st] = f(x)
                fd_g[i, k] = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
                fd_lap += (-vals[2] + 16 * vals[1] - 30 * l0 + 16 * vals[-1] - vals[-2]) / (12 * h * h)
        assert np.allclose(g[w].numpy(), fd_g, atol=1e-7)
        assert abs(float(lap[w]) - fd_lap) < 1e-5


def test_logdet_derivative_identities():
    """d log det / d Phi_ij = Phi^-1_ji and the Hessian -Phi^-1_jk Phi^-1_mi
    (Methods, efficient Laplacian) on random matrices, by central FD."""
    rng = np.random.default_rng(0)
    A = rng.normal(size=(5, 5))
    inv = np.linalg.inv(A)
    f = lambda X: np.linalg.slogdet(X)[1]
    h = 1e-5
    for (i, j) in [(0, 1), (3, 2), (4, 4)]:
        E = np.zeros_like(A)
        E[i, j] = h
        assert abs((f(A + E) - f(A - E)) / (2 * h) - inv[j, i]) < 1e-8
    h = 1e-4
    for (i, j, k, mm) in [(0, 1, 2, 3), (1, 1, 1, 1), (4, 0, 0, 2)]:
        Eij = np.zeros_like(A); Eij[i, j] = h
        Ekm = np.zeros_like(A); Ekm[k, mm] = h
        fd = (f(A + Eij + Ekm) - f(A + Eij - Ekm) - f(A - Eij + Ekm) + f(A - Eij - Ekm)) / (4 * h * h)
        assert abs(fd - (-inv[j, k] * inv[mm, i])) < 1e-6


def test_theta_gradient_vs_finite_differences():
    s, m, p, R = _orc(0, W=3)
    o = Oracle(s, m, p)
    coeff = np.array([0.7, -1.3, 0.4])
    g = o.grad_params(R, coeff)
    names = list(p.keys())
    rng = np.random.default_rng(5)
    for _ in range(6):
        dirs = {k: rng.normal(size=p[k].shape) for k in names}
        nrm = math.sqrt(sum((v ** 2).sum() for v in dirs.values()))
        dirs = {k: v / nrm for k, v in dirs.items()}
        h = 1e-5
        def val(t):
            q = {k: p[k] + t * dirs[k] for k in names}
            return float((Oracle(s, m, q).log_psi(R)[1].numpy() * coeff).sum())
        fd = (8 * (val(h) - val(-h)) - (val(2 * h) - val(-2 * h))) / (12 * h)
        an = sum(float((g[k].numpy() * dirs[k]).sum()) for k in names)
        assert abs(fd - an) < 1e-8 * max(1.0, abs(an))


# --------------------------------------------------------------------------
# determinant combination (Methods, eq. for Psi as a sum of determinants)
# --------------------------------------------------------------------------
def test_identical_determinants_add_log_k():
    s, m, p, R = _orc(0, W=3)
    o1 = Oracle(s, m, p)
    _, l1 = o1.log_psi(R)
    m3 = copy.deepcopy(m)
    m3.n_det = 3
    p3 = copy.deepcopy(p)
    for k in ("orb_W_up", "orb_W_dn", "env_pi_up", "env_pi_dn"):
        p3[k] = np.repeat(p[k], 3, axis=0)
    _, l3 = Oracle(s, m3, p3).log_psi(R)
    assert torch.allclose(l3, l1 + math.log(3), atol=1e-12, rtol=0)


def test_cancelling_determinants_give_sign_zero():
    s, m, p, R = _orc(0, W=2)
    m2 = copy.deepcopy(m)
    m2.n_det = 2
    p2 = copy.deepcopy(p)
    for k in ("orb_W_up", "orb_W_dn", "env_pi_up", "env_pi_dn"):
        p2[k] = np.repeat(p[k], 2, axis=0)
    p2["orb_W_up"][1][:, 0] *= -1.0          # flips the sign of det_2 (one column)
    sgn, _ = Oracle(s, m2, p2).log_psi(R)
    assert torch.all(sgn == 0)


# --------------------------------------------------------------------------
# potential (Methods, Hamiltonian) on hand-computed configurations
# --------------------------------------------------------------------------
def test_potential_hand_computed():
    R = np.array([[0.0, 0, 0], [0, 0, 2.0]])
    s = wl.make_system("HH", R, np.zeros(2, np.int32), pseudo_c=False)
    m = wl.make_model(s, width=4, mlp_layers=1, n_det=1, n_env=1)
    p = wl.init_params(s, m, np.random.default_rng(0))
    o = Oracle(s, m, p)
    el = np.array([[[0.0, 0, 1.0], [0.0, 3.0, 0]]])
    V = o.potential(el).numpy()[0]
    assert abs(V[0] - 1.0 / math.sqrt(1 + 9)) < 1e-14
    ven = -(1 / 1.0 + 1 / 1.0 + 1 / 3.0 + 1 / math.sqrt(9 + 4))
    assert abs(V[1] - ven) < 1e-14
    assert abs(V[2] - 0.5) < 1e-14
    # erf-smoothed local pseudopotential on a carbon with Z_eff = 4, width 0.5
    sC = wl.make_system("C", np.zeros((1, 3)), np.ones(1, np.int32), pseudo_c=True, n_up=2, n_dn=2)
    mC = wl.make_model(sC, width=4, mlp_layers=1, n_det=1, n_env=1)
    oC = Oracle(sC, mC, wl.init_params(sC, mC, np.random.default_rng(0)))
    el = np.array([[[0.3, 0, 0], [0, 1.0, 0], [0, 0, 2.0], [1.0, 1.0, 1.0]]])
    V = oC.potential(el).numpy()[0]
    rs = [0.3, 1.0, 2.0, math.sqrt(3)]
    assert abs(V[1] - sum(-4 * math.erf(r / 0.5) / r for r in rs)) < 1e-13
    assert V[2] == 0.0


# --------------------------------------------------------------------------
# pseudopotential quadrature (Methods, effective core potential)
# --------------------------------------------------------------------------
def test_icosahedron_is_a_spherical_5_design():
    from numpy.polynomial import legendre
    v = wl.icosahedron_vertices()
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    rng = np.random.default_rng(1)
    for _ in range(5):
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        c = v @ e
        for l in range(6):
            Pl = legendre.legval(c, [0] * l + [1])
            assert abs(Pl.mean() - (1.0 if l == 0 else 0.0)) < 1e-13


@pytest.mark.parametrize("nq,strength", [(4, 2), (6, 3), (12, 5)])
def test_quadrature_rules_are_spherical_designs(nq, strength):
    """The N_q-point rules (tetrahedron, octahedron, icosahedron) average
    P_l(e . e_q) to delta_l0 for every l up to their design strength and for
    any direction e, and not beyond it (so each rule is the one named)."""
    from numpy.polynomial import legendre
    from oracle import quadrature_directions
    v = quadrature_directions(nq).numpy()
    assert v.shape == (nq, 3) and np.allclose(np.linalg.norm(v, axis=1), 1.0, atol=1e-15)
    rng = np.random.default_rng(2)
    worst_next = 0.0
    for _ in range(6):
        e = rng.normal(size=3)
        e /= np.linalg.norm(e)
        c = v @ e
        for l in range(strength + 1):
            Pl = legendre.legval(c, [0] * l + [1])
            assert abs(Pl.mean() - (1.0 if l == 0 else 0.0)) < 1e-13
        worst_next = max(worst_next, abs(legendre.legval(c, [0] * (strength + 1) + [1]).mean()))
    assert worst_next > 1e-3


def test_icosahedron_rule_matches_the_generated_vertices():
    # two independent constructions of the 12-point set agree as point sets
    from oracle import quadrature_directions
    a = quadrature_directions(12).numpy()
    b = wl.icosahedron_vertices()
    d = np.linalg.norm(a[:, None] - b[None], axis=-1)
    assert np.allclose(d.min(1), 0.0, atol=1e-14) and np.allclose(d.min(0), 0.0, atol=1e-14)


@pytest.mark.parametrize("nq", [4, 6, 12])
def test_ecp_spherically_symmetric_wavefunction_gives_v0(nq):
    """With psi = exp(-r) centred on the pseudo-atom every ratio is 1 and the
    angular average of P_l vanishes for l = 1 under each rule: V_NL = v_0(r)."""
    s, m, p, R = wl.hydrogen_atom(W=5, seed=9)
    rng = np.random.default_rng(3)
    s.species = np.ones(1, np.int32)
    s.ecp = wl._ecp_tables(rng)
    s.ecp_nquad = {1: nq}
    R = R / np.linalg.norm(R, axis=-1, keepdims=True) * rng.uniform(0.2, 1.9, size=(5, 1, 1))
    o = Oracle(s, m, p)
    Q = wl.haar_rotations(5, rng)
    v = o.ecp_nonlocal(R, Q).numpy()
    r = np.linalg.norm(R[:, 0], axis=1)
    ch0 = s.ecp[1][0]
    v0 = (ch0.a[None] * np.exp(-ch0.alpha[None] * r[:, None] ** 2)).sum(1)
    assert np.allclose(v, v0, atol=1e-12)


@pytest.mark.parametrize("nq", [4, 6, 12])
@pytest.mark.parametrize("orient", ["along", "against"])
def test_ecp_p_type_wavefunction_gives_v1(nq, orient):
    """A p-type one-electron psi = (u . d) g(|d|) about the pseudo-atom, d =
    r - R_I, has quadrature ratios (u . q)/(u . dhat) with q the rotated rule
    direction.  Every rule of design strength >= 2 averages q q^T to I/3, so
    the l = 1 channel gives 3 (1/N_q) sum_q (dhat . q)(u . q)/(u . dhat) = 1
    and the l = 0 channel (1/N_q) sum_q (u . q)/(u . dhat) = 0: V_NL = v_1(r)
    exactly (the addition theorem for l = 1).  The case u . dhat < 0 makes
    every ratio's sign matter, and the Haar rotations Q make the Legendre
    argument depend on the rotated direction: a dropped (2l+1), P_1 taken on
    the unrotated rule or an unsigned ratio each break the equality."""
    s, m, p, R = wl.hydrogen_atom(W=6, seed=11)
    rng = np.random.default_rng(5)
    s.species = np.ones(1, np.int32)
    s.ecp = wl._ecp_tables(rng)
    s.ecp_nquad = {1: nq}
    dhat = rng.normal(size=(6, 3))
    dhat /= np.linalg.norm(dhat, axis=1, keepdims=True)
    r = rng.uniform(0.2, 1.9, size=6)
    R = (s.R_nuc[0][None] + dhat * r[:, None])[:, None, :]
    u = rng.normal(size=3)
    # choose the sign of u per case so that u . dhat has one sign on every walker
    dots = dhat @ u
    keep = np.abs(dots) > 0.2
    R, dhat, r, dots = R[keep], dhat[keep], r[keep], dots[keep]
    sgn = 1.0 if orient == "along" else -1.0
    R = R.copy()
    dhat = dhat * (np.sign(dots) * sgn)[:, None]
    R[:, 0] = s.R_nuc[0][None] + dhat * r[:, None]
    assert (np.sign(dhat @ u) == sgn).all()
    o = Oracle(s, m, p)
    Rn = torch.tensor(s.R_nuc[0])
    ut = torch.tensor(u)

    def p_type(X):
        X = torch.as_tensor(X, dtype=DT)
        d = X[:, 0] - Rn
        val = (d @ ut) * torch.exp(-0.7 * (d * d).sum(-1))
        return torch.sign(val), torch.log(val.abs())
    o.log_psi = p_type
    Q = wl.haar_rotations(len(R), rng)
    v = o.ecp_nonlocal(R, Q).numpy()
    ch1 = [c for c in s.ecp[1] if c.l == 1][0]
    v1 = (ch1.a[None] * np.exp(-ch1.alpha[None] * r[:, None] ** 2)).sum(1)
    assert np.allclose(v, v1, atol=1e-12, rtol=1e-12)
    # the test is not degenerate: the l = 1 value differs from v_0 and from 0
    ch0 = [c for c in s.ecp[1] if c.l == 0][0]
    v0 = (ch0.a[None] * np.exp(-ch0.alpha[None] * r[:, None] ** 2)).sum(1)
    assert np.abs(v1 - v0).min() > 1e-3 and np.abs(v1).min() > 1e-3


# --------------------------------------------------------------------------
# global single-electron jumps (SI, improved Monte Carlo sampling)
# --------------------------------------------------------------------------
def _gmm_oracle(name):
    if name == "h2":
        R, sp = wl.h_chain(2, spacing=1.4)
        s = wl.make_system("H2", R, sp, pseudo_c=False)
    else:
        R, sp = wl.cumulene(2)
        s = wl.make_system("C2H4", R, sp, pseudo_c=True)
    m = wl.make_model(s, width=8, mlp_layers=1, n_det=1, n_env=1, cutoff=3.0, cutoff_nuc=20.0)
    return Oracle(s, m, wl.init_params(s, m, np.random.default_rng(0))), s


@pytest.mark.parametrize("name", ["h2", "c2h4"])
def test_gmm_density_is_normalised(name):
    """rho_global is a probability density: a 3D grid quadrature (spacing
    0.25 bohr, spectrally accurate for Gaussians of width 2) integrates it
    to 1."""
    o, s = _gmm_oracle(name)
    lo, hi = s.R_nuc.min(0) - 16.0, s.R_nuc.max(0) + 16.0
    h = 0.25
    axes = [torch.arange(lo[k], hi[k] + h / 2, h, dtype=DT) for k in range(3)]
    tot = 0.0
    for x in axes[0]:
        Y, Z = torch.meshgrid(axes[1], axes[2], indexing="ij")
        pts = torch.stack([torch.full_like(Y, float(x)), Y, Z], -1)
        tot += float(torch.exp(o.gmm_log_density(pts, 2.0)).sum()) * h ** 3
    assert abs(tot - 1.0) < 1e-6


def test_gmm_density_single_nucleus_closed_form():
    # one nucleus: rho is N(R, tau^2 I); at R it is (2 pi tau^2)^(-3/2)
    s, m, p, _ = wl.hydrogen_atom(W=1, seed=0)
    o = Oracle(s, m, p)
    for tau in (0.5, 2.0, 3.0):
        r = torch.tensor([[0.0, 0.0, 0.0], [1.0, -2.0, 0.5]], dtype=DT)
        got = o.gmm_log_density(r, tau).numpy()
        want = -1.5 * math.log(2 * math.pi * tau * tau) - np.array([0.0, 5.25]) / (2 * tau * tau)
        assert np.allclose(got, want, atol=1e-14, rtol=0)


def test_gmm_draw_component_weights():
    """Component m is drawn with probability Z_m / sum Z: uniform picks on a
    fine grid land on each nucleus in that proportion, and with xi = 0 the
    draw is the nucleus itself."""
    o, s = _gmm_oracle("c2h4")
    K = 60000
    pick = (torch.arange(K, dtype=DT) + 0.5) / K
    r = o.gmm_draw(pick, torch.zeros(K, 3, dtype=DT), 2.0)
    d = torch.cdist(r, torch.tensor(s.R_nuc, dtype=DT))
    assert float(d.min(1).values.max()) == 0.0
    counts = np.bincount(d.argmin(1).numpy(), minlength=len(s.Z)) / K
    assert np.allclose(counts, s.Z / s.Z.sum(), atol=2.0 / K)
    # xi moves the draw by tau xi
    xi = torch.tensor([[0.3, -1.0, 2.0]], dtype=DT)
    r1 = o.gmm_draw(torch.tensor([0.0], dtype=DT), xi, 2.0)
    assert torch.allclose(r1[0], torch.tensor(s.R_nuc[0], dtype=DT) + 2.0 * xi[0], atol=0, rtol=0)


def test_hydrogen_sampling_with_global_jumps():
    """Only global jumps (an independence sampler from N(0, 4 I)) and
    alternating local/global sweeps both sample |psi|^2 = exp(-2r)/pi:
    <r> = 3/2.  Without the proposal factor the chain would instead sample
    |psi|^2 rho (detailed balance of the uncorrected independence sampler),
    whose mean radius is computed here and lies far outside the tolerance."""
    s, m, p, R0 = wl.hydrogen_atom(W=512, seed=6)
    o = Oracle(s, m, p)
    r = np.linspace(0.0, 40.0, 400001)
    wt = r ** 2 * np.exp(-2.0 * r - r ** 2 / 8.0)
    biased = float((r * wt).sum() / wt.sum())
    assert abs(biased - 1.5) > 0.2
    for kinds in ([1] * 10, [0, 1] * 5):
        rng = np.random.default_rng(12)
        R = R0 * 0.5
        rs = []
        for blk in range(30):
            xi, u = wl.mcmc_noise(10, 1, 512, rng)
            pk = rng.uniform(size=u.shape)
            R, _, _, _ = o.mcmc_sweep(R, 1.0, xi, u, kinds=kinds, pick=pk, gstep=2.0)
            if blk >= 8:
                rs.append(np.linalg.norm(R.numpy()[:, 0], axis=1).mean())
        assert abs(np.mean(rs) - 1.5) < 0.03


# --------------------------------------------------------------------------
# cusp Jastrow factor (Methods, global electron correlation)
# --------------------------------------------------------------------------
def test_jastrow_cusp_closed_form_and_cusp_conditions():
    """log psi gains sum_{i<j} w a^2/(a + r_ij) per spin class: checked on H4
    against the pair sum written from the positions, and the slope at
    coalescence is -w: with w_par = -1/4, w_anti = -1/2 the Kato cusp
    conditions d(log psi)/dr = 1/4 (equal spins) and 1/2 (opposite spins)."""
    s, m, p, R = _orc(0, W=3)
    o0 = Oracle(s, m, copy.deepcopy(p))
    q = np.array([-0.25, 0.7, -0.5, 1.3])
    p1 = copy.deepcopy(p)
    p1["jas_cusp"] = q.copy()
    o1 = Oracle(s, m, p1)
    _, l0 = o0.log_psi(R)
    _, l1 = o1.log_psi(R)
    spin = np.arange(s.n_el) >= s.n_up
    want = np.zeros(R.shape[0])
    for i in range(s.n_el):
        for j in range(i + 1, s.n_el):
            r = np.linalg.norm(R[:, i] - R[:, j], axis=1)
            w, a = (q[0], q[1]) if spin[i] == spin[j] else (q[2], q[3])
            want += w * a * a / (a + r)
    assert np.allclose((l1 - l0).numpy(), want, atol=1e-12, rtol=0)
    # slope of J along r_12 at coalescence for a lone pair: -w
    Rh, sp = wl.h_chain(2, spacing=1.4)
    for (nu, nd, slope) in ((2, 0, 0.25), (1, 1, 0.5)):
        s2 = wl.make_system("H2", Rh, sp, pseudo_c=False, n_up=nu, n_dn=nd)
        m2 = wl.make_model(s2, width=8, mlp_layers=1, n_det=1, n_env=1, cutoff=3.0, cutoff_nuc=20.0)
        p2 = wl.init_params(s2, m2, np.random.default_rng(0))
        p2["jas_cusp"] = np.array([-0.25, 0.8, -0.5, 1.2])
        o2 = Oracle(s2, m2, p2)
        hs = 1e-7
        x = np.zeros((2, 2, 3))
        x[:, 0] = [0.3, -0.2, 0.1]
        x[0, 1] = x[0, 0] + [hs, 0.0, 0.0]
        x[1, 1] = x[1, 0] + [2 * hs, 0.0, 0.0]
        jv = o2.jastrow_cusp(x).numpy()
        assert abs((jv[1] - jv[0]) / hs - slope) < 1e-5


def test_jastrow_is_symmetric_and_zero_by_default():
    s, m, p, R = _orc(0, W=2)
    assert np.array_equal(p["jas_cusp"], [0.0, 1.0, 0.0, 1.0])
    o = Oracle(s, m, p)
    assert float(o.jastrow_cusp(R).abs().max()) == 0.0
    p1 = copy.deepcopy(p)
    p1["jas_cusp"] = np.array([-0.3, 0.9, -0.45, 1.1])
    o1 = Oracle(s, m, p1)
    Rs = R.copy()
    Rs[:, [0, 1]] = Rs[:, [1, 0]]          # same-spin swap
    Rs[:, [2, 3]] = Rs[:, [3, 2]]
    assert torch.allclose(o1.jastrow_cusp(R), o1.jastrow_cusp(Rs), atol=1e-14, rtol=0)


# --------------------------------------------------------------------------
# MLP Jastrow (Methods, global electron correlation: exp(sum_i MLP_1(h_i))
# times sum_i MLP_2(h_i) over the final embeddings)
# --------------------------------------------------------------------------
def _silu_np(x):
    return x / (1.0 + np.exp(-x))


def _jmlp_h4(W=3, Hj=8, seed=11):
    s, m, p, R = _orc(0, W=W)
    m.jas_mlp_width = Hj
    p = wl.init_params(s, m, np.random.default_rng(seed))
    m0 = copy.deepcopy(m)
    m0.jas_mlp_width = 0
    p0 = {k: v for k, v in p.items() if not k.startswith("jmlp_")}
    return s, m, p, m0, p0, R


def test_jastrow_mlp_constant_readouts_closed_form():
    """With W1 = W2 = 0 every readout is the constant c_k = w3_k . SiLU(b2_k)
    + b3_k, so log|psi| gains n c_1 + log|n c_2| and the sign takes
    sign(c_2), for either sign of c_2."""
    s, m, p, m0, p0, R = _jmlp_h4()
    s0, l0 = Oracle(s, m0, p0).log_psi(R)
    q = copy.deepcopy(p)
    q["jmlp_W1"][:] = 0.0
    q["jmlp_W2"][:] = 0.0
    q["jmlp_b2"] = np.random.default_rng(3).normal(size=q["jmlp_b2"].shape)
    n = s.n_el
    for b3 in ([0.3, 0.2], [-0.1, -0.9]):
        q["jmlp_b3"] = np.array(b3)
        c = [float(np.dot(q["jmlp_w3"][k], _silu_np(q["jmlp_b2"][k]))) + b3[k] for k in (0, 1)]
        s1, l1 = Oracle(s, m, q).log_psi(R)
        assert np.allclose((l1 - l0).numpy(), n * c[0] + math.log(abs(n * c[1])), atol=1e-12, rtol=0)
        assert np.array_equal(s1.numpy(), s0.numpy() * np.sign(c[1]))


def test_jastrow_mlp_single_path_hand_computed():
    """One live path per readout: W1_k = v_k e_0^T (a column of the [d][Hj]
    matrix), W2_k = a_k e_0 e_1^T (hidden unit 0 feeds unit 1), so MLP_k(h) =
    w3_k[1] SiLU(a_k SiLU(h . v_k + b1_k[0]) + b2_k[1]) + sum_{c != 1}
    w3_k[c] SiLU(b2_k[c]) + b3_k, summed over the final embeddings h_i; a
    transposed layer, swapped readouts or a dropped log fail it."""
    s, m, p, m0, p0, R = _jmlp_h4(W=4)
    rng = np.random.default_rng(8)
    q = copy.deepcopy(p)
    d, Hj = m.width, m.jas_mlp_width
    v = rng.normal(size=(2, d)) / math.sqrt(d)
    a = np.array([1.3, -0.8])
    q["jmlp_W1"] = np.zeros((2, d, Hj))
    q["jmlp_W2"] = np.zeros((2, Hj, Hj))
    for k in (0, 1):
        q["jmlp_W1"][k, :, 0] = v[k]
        q["jmlp_W2"][k, 0, 1] = a[k]
    q["jmlp_b1"] = rng.normal(size=(2, Hj))
    q["jmlp_b2"] = rng.normal(size=(2, Hj))
    q["jmlp_b3"] = np.array([0.2, 0.5])
    o = Oracle(s, m, q)
    h = o.embed(torch.as_tensor(R))["h"].numpy()                # [B, n, d]
    S = []
    for k in (0, 1):
        w3, b1, b2 = q["jmlp_w3"][k], q["jmlp_b1"][k], q["jmlp_b2"][k]
        live = w3[1] * _silu_np(a[k] * _silu_np(h @ v[k] + b1[0]) + b2[1])
        dead = float(np.dot(w3, _silu_np(b2))) - w3[1] * _silu_np(b2[1])
        S.append((live + dead + q["jmlp_b3"][k]).sum(1))
    _, l0 = Oracle(s, m0, p0).log_psi(R)
    s1, l1 = o.log_psi(R)
    assert np.allclose((l1 - l0).numpy(), S[0] + np.log(np.abs(S[1])), atol=1e-12, rtol=0)
    s0, _ = Oracle(s, m0, p0).log_psi(R)
    assert np.array_equal(s1.numpy(), s0.numpy() * np.sign(S[1]))


def test_jastrow_mlp_is_symmetric_under_same_spin_swaps():
    """The factor is symmetric, so log|psi| keeps its value and the sign
    flips under a same-spin exchange, as without it."""
    s, m, p, m0, p0, R = _jmlp_h4()
    o = Oracle(s, m, p)
    Rs = R.copy()
    Rs[:, [0, 1]] = Rs[:, [1, 0]]
    sa, la = o.log_psi(R)
    sb, lb = o.log_psi(Rs)
    assert torch.allclose(la, lb, atol=1e-12, rtol=0)
    assert torch.equal(sa, -sb)


def test_jastrow_mlp_gradient_and_laplacian_vs_finite_differences():
    """grad and Lap of log|psi| with the MLP Jastrow (autodiff in the oracle)
    against fourth-order central differences of log|psi| itself."""
    s, m, p, m0, p0, R = _jmlp_h4(W=2)
    o = Oracle(s, m, p)
    g, lap = o.grad_lap(R)
    h = 1e-3
    for w in range(2):
        x0 = R[w].copy()
        f = lambda x: float(o.log_psi(x[None])[1][0])
        l0 = f(x0)
        fd_lap, fd_g = 0.0, np.zeros_like(x0)
        for i in range(s.n_el):
            for k in range(3):
                vals = {}
                for st in (-2, -1, 1, 2):
                    x = x0.copy()
                    x[i, k] += st * h
                    vals[st] = f(x)
                fd_g[i, k] = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
                fd_lap += (-vals[2] + 16 * vals[1] - 30 * l0 + 16 * vals[-1] - vals[-2]) / (12 * h * h)
        assert np.allclose(g[w].numpy(), fd_g, atol=1e-7 * max(1.0, np.abs(fd_g).max()))
        # fourth-order differences: relative error ~1e-7 at |Lap| of several hundred
        assert abs(float(lap[w]) - fd_lap) < 1e-6 * max(1.0, abs(fd_lap))


def test_jastrow_mlp_theta_gradient_vs_finite_differences():
    s, m, p, m0, p0, R = _jmlp_h4(W=3)
    o = Oracle(s, m, p)
    coeff = np.array([0.7, -1.3, 0.4])
    g = o.grad_params(R, coeff)
    names = [k for k in p if k.startswith("jmlp_")] + ["mlp_W", "glu_Wo"]
    rng = np.random.default_rng(6)
    for _ in range(4):
        dirs = {k: rng.normal(size=p[k].shape) for k in names}
        nrm = math.sqrt(sum((v ** 2).sum() for v in dirs.values()))
        dirs = {k: v / nrm for k, v in dirs.items()}
        hh = 1e-5

        def val(t):
            q = dict(p)
            for k in names:
                q[k] = p[k] + t * dirs[k]
            return float((Oracle(s, m, q).log_psi(R)[1].numpy() * coeff).sum())
        fd = (8 * (val(hh) - val(-hh)) - (val(2 * hh) - val(-2 * hh))) / (12 * hh)
        an = sum(float((g[k].numpy() * dirs[k]).sum()) for k in names)
        assert abs(fd - an) < 1e-8 * max(1.0, abs(an))


# --------------------------------------------------------------------------
# attention Jastrow (Methods, global electron correlation: cross attention of
# register queries over the electron embeddings, exp(MLP_1(V)) MLP_2(V))
# --------------------------------------------------------------------------
def _jatt_h4(W=3, regs=4, dr=4, Ha=8, seed=12):
    s, m, p, R = _orc(0, W=W)
    m.jas_att_regs, m.jas_att_dim, m.jas_att_width = regs, dr, Ha
    p = wl.init_params(s, m, np.random.default_rng(seed))
    m0 = copy.deepcopy(m)
    m0.jas_att_regs = 0
    p0 = {k: v for k, v in p.items() if not k.startswith("jatt_")}
    return s, m, p, m0, p0, R


def _single_path_readout(q, rng, width, Ha):
    """Readouts with one live path each (as in the MLP Jastrow pin): returns
    the live directions v_k and gains a_k."""
    v = rng.normal(size=(2, width)) / math.sqrt(width)
    a = np.array([1.1, -0.7])
    q["jatt_W1"] = np.zeros((2, width, Ha))
    q["jatt_W2"] = np.zeros((2, Ha, Ha))
    for k in (0, 1):
        q["jatt_W1"][k, :, 0] = v[k]
        q["jatt_W2"][k, 0, 1] = a[k]
    q["jatt_b1"] = rng.normal(size=(2, Ha))
    q["jatt_b2"] = rng.normal(size=(2, Ha))
    q["jatt_b3"] = np.array([0.3, -0.6])
    return v, a


def _readout_np(q, V, v, a):
    out = []
    for k in (0, 1):
        w3, b1, b2 = q["jatt_w3"][k], q["jatt_b1"][k], q["jatt_b2"][k]
        live = w3[1] * _silu_np(a[k] * _silu_np(V @ v[k] + b1[0]) + b2[1])
        dead = float(np.dot(w3, _silu_np(b2))) - w3[1] * _silu_np(b2[1])
        out.append(live + dead + q["jatt_b3"][k])
    return out


def test_jastrow_att_uniform_attention_closed_form():
    """Zero queries make every softmax uniform: v_r = mean_i h_i W^V_r, and
    with single-path readouts log|J_att| = MLP_1(V) + log|MLP_2(V)| follows
    by hand; the register order (r-major concatenation) and the value-map
    orientation are fixed by it."""
    s, m, p, m0, p0, R = _jatt_h4(W=4)
    rng = np.random.default_rng(4)
    q = copy.deepcopy(p)
    q["jatt_q"][:] = 0.0
    regs, dr = m.jas_att_regs, m.jas_att_dim
    v, a = _single_path_readout(q, rng, regs * dr, m.jas_att_width)
    o = Oracle(s, m, q)
    h = o.embed(torch.as_tensor(R))["h"].numpy()
    V = np.concatenate([h.mean(1) @ q["jatt_Wv"][r] for r in range(regs)], axis=1)
    o1, o2 = _readout_np(q, V, v, a)
    _, l0 = Oracle(s, m0, p0).log_psi(R)
    s0, _ = Oracle(s, m0, p0).log_psi(R)
    s1, l1 = o.log_psi(R)
    assert np.allclose((l1 - l0).numpy(), o1 + np.log(np.abs(o2)), atol=1e-12, rtol=0)
    assert np.array_equal(s1.numpy(), s0.numpy() * np.sign(o2))


def test_jastrow_att_sharp_attention_limit():
    """Queries scaled by a large factor make each softmax pick the electron
    with the largest logit h_i . q_r: v_r -> h_{i*} W^V_r."""
    s, m, p, m0, p0, R = _jatt_h4(W=4)
    rng = np.random.default_rng(9)
    q = copy.deepcopy(p)
    regs, dr = m.jas_att_regs, m.jas_att_dim
    v, a = _single_path_readout(q, rng, regs * dr, m.jas_att_width)
    q["jatt_q"] = q["jatt_q"] * 1.0e4
    o = Oracle(s, m, q)
    h = o.embed(torch.as_tensor(R))["h"].numpy()
    lg = np.einsum("bnd,rd->bnr", h, q["jatt_q"])
    srt = np.sort(lg, axis=1)
    assert (srt[:, -1] - srt[:, -2]).min() > 40.0        # the runner-up weight is below e^-40
    top = lg.argmax(1)                                     # [B, regs]
    V = np.concatenate([h[np.arange(h.shape[0]), top[:, r]] @ q["jatt_Wv"][r] for r in range(regs)], axis=1)
    Vo = o.jastrow_att_registers(torch.as_tensor(h)).numpy()
    assert np.allclose(Vo, V, atol=1e-12, rtol=0)
    o1, o2 = _readout_np(q, V, v, a)
    _, l0 = Oracle(s, m0, p0).log_psi(R)
    _, l1 = o.log_psi(R)
    assert np.allclose((l1 - l0).numpy(), o1 + np.log(np.abs(o2)), atol=1e-10, rtol=0)


def test_jastrow_att_weak_attention_slope():
    """At queries lambda q the register embedding's slope at lambda = 0 is
    the covariance over the electrons of the logit h_i . q_r and the value
    h_i W^V_r (the first-order expansion of the softmax about uniform
    weights): dv_r/dlambda = mean_i (l_ri - mean l_r) u_ri."""
    s, m, p, m0, p0, R = _jatt_h4(W=3)
    o = Oracle(s, m, p)
    h = o.embed(torch.as_tensor(R))["h"]
    qhat = p["jatt_q"].copy()
    regs = m.jas_att_regs
    lam = 1e-4
    Vs = []
    for t in (lam, -lam):
        o.p["jatt_q"] = torch.as_tensor(t * qhat)
        Vs.append(o.jastrow_att_registers(h).numpy())
    slope = (Vs[0] - Vs[1]) / (2 * lam)
    hn = h.numpy()
    want = []
    for r in range(regs):
        lg = hn @ qhat[r]                                   # [B, n]
        u = hn @ p["jatt_Wv"][r]                            # [B, n, dr]
        want.append(((lg - lg.mean(1, keepdims=True))[..., None] * u).mean(1))
    want = np.concatenate(want, axis=1)
    assert np.abs(slope - want).max() <= 1e-6 * max(1.0, np.abs(want).max())


def test_jastrow_att_gradient_and_laplacian_vs_finite_differences():
    s, m, p, m0, p0, R = _jatt_h4(W=2)
    o = Oracle(s, m, p)
    g, lap = o.grad_lap(R)
    h = 1e-3
    for w in range(2):
        x0 = R[w].copy()
        f = lambda x: float(o.log_psi(x[None])[1][0])
        l0 = f(x0)
        fd_lap, fd_g = 0.0, np.zeros_like(x0)
        for i in range(s.n_el):
            for k in range(3):
                vals = {}
                for st in (-2, -1, 1, 2):
                    x = x0.copy()
                    x[i, k] += st * h
                    vals[st] = f(x)
                fd_g[i, k] = (8 * (vals[1] - vals[-1]) - (vals[2] - vals[-2])) / (12 * h)
                fd_lap += (-vals[2] + 16 * vals[1] - 30 * l0 + 16 * vals[-1] - vals[-2]) / (12 * h * h)
        assert np.allclose(g[w].numpy(), fd_g, atol=1e-7 * max(1.0, np.abs(fd_g).max()))
        assert abs(float(lap[w]) - fd_lap) < 1e-6 * max(1.0, abs(fd_lap))


def test_jastrow_att_theta_gradient_vs_finite_differences():
    s, m, p, m0, p0, R = _jatt_h4(W=3)
    o = Oracle(s, m, p)
    coeff = np.array([0.7, -1.3, 0.4])
    g = o.grad_params(R, coeff)
    names = [k for k in p if k.startswith("jatt_")] + ["mlp_W"]
    rng = np.random.default_rng(6)
    for _ in range(4):
        dirs = {k: rng.normal(size=p[k].shape) for k in names}
        nrm = math.sqrt(sum((v ** 2).sum() for v in dirs.values()))
        dirs = {k: v / nrm for k, v in dirs.items()}
        hh = 1e-5

        def val(t):
            q = dict(p)
            for k in names:
                q[k] = p[k] + t * dirs[k]
            return float((Oracle(s, m, q).log_psi(R)[1].numpy() * coeff).sum())
        fd = (8 * (val(hh) - val(-hh)) - (val(2 * hh) - val(-2 * hh))) / (12 * hh)
        an = sum(float((g[k].numpy() * dirs[k]).sum()) for k in names)
        assert abs(fd - an) < 1e-8 * max(1.0, abs(an))


# --------------------------------------------------------------------------
# the counter-based generator of the sampler's own random numbers
# --------------------------------------------------------------------------
def test_philox_known_answer_vectors():
    """Philox4x32-10 reproduces the published known-answer vectors."""
    import os
    from oracle.philox import philox4x32_10
    path = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")
    rows = [l.split() for l in open(path) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        out = philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in out] == v[6:10]


def test_sweep_randoms_distribution():
    """The Metropolis draws: uniforms inside (0, 1) with mean 1/2 and
    variance 1/12, normals with mean 0, variance 1 and kurtosis 3 (within
    five standard errors over 2^17 draws); different sweeps, electrons and
    walkers give different numbers."""
    from oracle.philox import sweep_randoms
    xi, u = sweep_randoms(12345, 7, 0, 128, 1024)
    assert xi.shape == (128, 1024, 3) and u.shape == (128, 1024)
    assert (u > 0).all() and (u < 1).all()
    N = u.size
    assert abs(u.mean() - 0.5) < 5 * np.sqrt(1 / 12 / N)
    assert abs(u.var() - 1 / 12) < 5 * np.sqrt(1 / 180 / N)
    z = xi.reshape(-1)
    assert abs(z.mean()) < 5 / np.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    assert abs((z ** 4).mean() - 3.0) < 5 * np.sqrt(96.0 / z.size)
    xi2, u2 = sweep_randoms(12345, 7, 1, 128, 1024)
    assert not np.any(u2 == u)
    assert len(np.unique(u)) == u.size


# --------------------------------------------------------------------------
# the natural-gradient step (Methods, variational Monte Carlo, eq. spring;
# SI, non-hermitian operator gradients in Spring, eq. aux_spring)
# --------------------------------------------------------------------------
def _spring_data(W=12, P=30, seed=0):
    rng = np.random.default_rng(seed)
    O = rng.normal(size=(W, P)) + 0.3 * rng.normal(size=P)
    e = rng.normal(size=W) * 2.0 - 5.0
    dprev = rng.normal(size=P) * 0.1
    return O, e, dprev


def test_spring_is_the_damped_least_squares_minimiser():
    """delta minimises |Obar delta - eps|^2 + lam |delta - eta delta_prev|^2:
    it equals the P x P normal-equation solution (Obar^T Obar + lam I)^-1
    (Obar^T eps + lam eta delta_prev), and the objective's gradient vanishes
    there (Obar, eps centred over the walkers)."""
    from oracle import spring_step
    O, e, dprev = _spring_data()
    lam, eta = 0.05, 0.9
    d = spring_step(O, e, lam, eta, dprev)
    Ob = O - O.mean(0)
    eps = e - e.mean()
    P = O.shape[1]
    ref = np.linalg.solve(Ob.T @ Ob + lam * np.eye(P), Ob.T @ eps + lam * eta * dprev)
    assert np.allclose(d, ref, rtol=1e-10, atol=1e-12)
    grad = Ob.T @ (Ob @ d - eps) + lam * (d - eta * dprev)
    assert np.abs(grad).max() < 1e-10 * max(1.0, np.abs(Ob.T @ eps).max())


def test_spring_interpolates_as_damping_vanishes():
    """With W - 1 <= P the centred Gram matrix has full rank on the centred
    vectors, so as lam -> 0 the update reproduces the centred energies:
    Obar delta -> eps (momentum off)."""
    from oracle import spring_step
    O, e, _ = _spring_data(W=10, P=40, seed=1)
    d = spring_step(O, e, 1e-10, 0.0)
    Ob = O - O.mean(0)
    assert np.abs(Ob @ d - (e - e.mean())).max() < 1e-6


def test_spring_extra_gradient_split():
    """An extra gradient in the span of the rows of Obar is carried entirely
    through eps (its out-of-span rest vanishes), one orthogonal to every row
    passes through unchanged, and without one the update is eq. spring."""
    from oracle import spring_step
    O, e, dprev = _spring_data(W=8, P=25, seed=2)
    lam, eta = 1e-2, 0.99
    Ob = O - O.mean(0)
    base = spring_step(O, e, lam, eta, dprev)
    # orthogonal to every row of Obar: eps~ = 0
    rng = np.random.default_rng(3)
    v = rng.normal(size=O.shape[1])
    Q, _ = np.linalg.qr(Ob.T)
    v_out = v - Q @ (Q.T @ v)
    d_out = spring_step(O, e, lam, eta, dprev, delta_tilde=v_out, lam_pinv=1e-12)
    assert np.allclose(d_out, base + v_out, atol=1e-10)
    # in the span: delta~ = Obar^T a; then the rest vanishes and eps~ = the
    # centred a (the pseudo-inverse solution on the range)
    a = rng.normal(size=O.shape[0])
    v_in = Ob.T @ a
    d_in = spring_step(O, e, lam, eta, dprev, delta_tilde=v_in, lam_pinv=1e-12)
    a_c = a - a.mean()
    x = np.linalg.solve(Ob @ Ob.T + lam * np.eye(O.shape[0]), (e - e.mean()) + a_c - Ob @ (eta * dprev))
    assert np.allclose(d_in, Ob.T @ x + eta * dprev, atol=1e-8)


# --------------------------------------------------------------------------
# S+ spin penalty (SI, low-rank updates in S+ operator)
# --------------------------------------------------------------------------
def _closed_shell_h4(W=6, seed=4, n_det=2):
    """H4 (2 up, 2 down) with the zeroed network (every embedding the same
    constant) and the same orbital weights and envelopes in both spin blocks:
    every determinant is a closed-shell product D(phi; r_up) D(phi; r_down)
    of one set of spatial orbitals."""
    w = wl.config(0, walkers=W)
    s, m, p, R = w.systems[0], w.model, w.params[0], w.R[0]
    m.n_det = n_det
    rng = np.random.default_rng(seed)
    p = wl.init_params(s, m, rng)
    wl.zero_network(p)
    p["orb_W_dn"] = p["orb_W_up"].copy()
    p["env_pi_dn"] = p["env_pi_up"].copy()
    return s, m, p, R


def test_splus_estimator_vanishes_for_closed_shell_products():
    """For a sum of closed-shell products, each factor built from one set of
    spatial orbitals for both spins, sum_a psi(pi_{a,beta} r)/psi(r) = 1 at
    every configuration (expanding the swapped determinants by their rows:
    sum_a sum_k phi_k(r_beta) (Phi_up^-1)_ka phi_l(r_a) (Phi_dn^-1)_lb
    collapses through Phi_up^-1 Phi_up = I to (Phi_dn Phi_dn^-1)_bb = 1), so
    R_beta = 0: the singlet has no S+ component.  With different orbitals in
    the two blocks it does not vanish."""
    s, m, p, R = _closed_shell_h4()
    o = Oracle(s, m, p)
    for beta in (2, 3):
        ratios, rb = o.splus_ratios(R, beta)
        assert np.abs(rb.numpy()).max() < 1e-10
        assert np.abs(ratios.numpy()).max() > 1e-3     # the ratios themselves are not trivial
    p2 = dict(p)
    p2["env_pi_dn"] = p["env_pi_dn"] + 0.5 * np.random.default_rng(8).normal(size=p["env_pi_dn"].shape)
    _, rb2 = Oracle(s, m, p2).splus_ratios(R, 2)
    assert np.abs(rb2.numpy()).min() > 1e-6


def test_splus_swap_is_an_involution():
    """Swapping twice restores the configuration: the ratio at the swapped
    walkers is the reciprocal of the ratio at the original ones."""
    w = wl.config(0, walkers=5)
    o = Oracle(w.systems[0], w.model, w.params[0])
    R = w.R[0]
    r1, _ = o.splus_ratios(R, 2)
    Rs = R.copy()
    Rs[:, [0, 2]] = R[:, [2, 0]]
    r2, _ = o.splus_ratios(Rs, 2)
    assert np.allclose(r1[:, 0].numpy() * r2[:, 0].numpy(), 1.0, rtol=1e-12)
