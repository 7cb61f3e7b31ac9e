"""Plain FP64 CPU oracle of the FiRE hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU leg of
the benchmark may import this module; the product path never does.

It is the dense definition of the method, evaluated walker-batched with
torch float64 on the CPU:

* every electron pair and every electron-nucleus pair is evaluated; the
  cutoffs enter only through the smooth cutoff factor, which is exactly zero
  at and beyond the cutoff, so the sum over all pairs equals the sum over the
  finite-range neighbourhoods (Methods, "Finite-range embeddings");
* every Metropolis proposal and every pseudopotential quadrature point is a
  full re-evaluation (no low-rank update);
* gradients, Laplacians and parameter gradients come from reverse/forward
  automatic differentiation, not from the sparse forward Laplacian.

Readings of the paper where it is silent (all listed in the design notes):
spin-block determinants; exp(-sigma |r - R|) envelopes with exponents shared
over orbitals; SiLU activations; a LLaMA-style GLU W_o[(LN(s)W_v+b_v) *
SiLU(LN(s)W_g+b_g)] + b_o; filters 4 -> 16 -> 8 -> d with a 32-Gaussian radial
part; the polynomial cutoff with p = 6; separate parallel/antiparallel
message weights; of the Jastrow terms the cusp factor, exp of a pair sum
with (w, a) per spin class (zero weights by default), and optionally the
per-electron MLP factor exp(sum_i MLP_1(h_i)) sum_i MLP_2(h_i) over the final
embeddings and the attention factor exp(MLP_1(V)) MLP_2(V) over register
embeddings V (softmax over the electrons of h_i . q_r weighting h_i W^V_r),
each MLP two SiLU hidden layers and a scalar linear readout, the factors
multiplying (their logs add); semilocal l = 0, 1 pseudopotential
channels with an equal-weight angular rule per species (12-point icosahedron
unless the system names 4 or 6 points).

The paper prints no worked example for this path, so no function here is
compared with a printed number; every function is pinned instead by the
identities, limits, closed forms and brute-force checks in
tests/test_oracle_pins.py (each test names the function it pins).
"""
from __future__ import annotations

import math
from typing import Dict, Optional

import numpy as np
import torch

torch.set_default_dtype(torch.float64)
DT = torch.float64
FCUT_P = 6
LN_EPS = 1e-5


def silu(x):
    return x * torch.sigmoid(x)


def fcut(x):
    """Polynomial cutoff of Gasteiger et al. with p = 6 (Methods, spatial
    filters): 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2) below
    x = 1, exactly zero at and beyond 1."""
    p = FCUT_P
    poly = 1 - (p + 1) * (p + 2) / 2 * x ** p + p * (p + 2) * x ** (p + 1) - p * (p + 1) / 2 * x ** (p + 2)
    return torch.where(x < 1.0, poly, torch.zeros_like(x))


def _safe_norm(v, mask_zero=None):
    """|v| along the last axis; entries flagged in mask_zero are computed on a
    dummy unit vector so autodiff never sees the singular point (they are
    multiplied by zero by the caller)."""
    if mask_zero is not None:
        dummy = torch.zeros_like(v)
        dummy[..., 0] = 1.0
        v = torch.where(mask_zero[..., None], dummy, v)
    return torch.sqrt((v * v).sum(-1)), v


def _log1p_over(r):
    """log(1+r)/r with its limit 1 at r = 0."""
    small = r < 1e-8
    rs = torch.where(small, torch.ones_like(r), r)
    return torch.where(small, 1.0 - 0.5 * r, torch.log1p(rs) / rs)


def quadrature_directions(n_quad: int) -> torch.Tensor:
    """Unit vectors of the equal-weight angular quadrature with n_quad points
    (SI, effective core potential, N_quad per species): the vertices of the
    tetrahedron (4), octahedron (6) or icosahedron (12), spherical designs of
    strength 2, 3 and 5."""
    if n_quad == 4:
        v = np.array([[1, 1, 1], [1, -1, -1], [-1, 1, -1], [-1, -1, 1]], float) / math.sqrt(3.0)
    elif n_quad == 6:
        v = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    elif n_quad == 12:
        ph = (1.0 + math.sqrt(5.0)) / 2.0
        v = []
        for a in (1.0, -1.0):
            for b in (ph, -ph):
                v += [[0.0, a, b], [a, b, 0.0], [b, 0.0, a]]
        v = np.array(v) / math.sqrt(1.0 + ph * ph)
    else:
        raise ValueError(f"no {n_quad}-point rule")
    return torch.tensor(v, dtype=DT)


class Oracle:
    """Dense FP64 evaluation of one system with one parameter set."""

    def __init__(self, system, model, params: Dict[str, np.ndarray]):
        self.sys = system
        self.model = model
        self.n_up, self.n_dn = system.n_up, system.n_dn
        self.n = system.n_el
        self.Rn = torch.tensor(system.R_nuc, dtype=DT)
        self.Z = torch.tensor(system.Z, dtype=DT)
        self.nuc_type = torch.tensor(system.nuc_type, dtype=torch.long)
        self.pp_width = torch.tensor(system.pp_width, dtype=DT)
        self.p = {k: torch.tensor(v, dtype=DT) for k, v in params.items()}
        spin = torch.zeros(self.n, dtype=torch.long)
        spin[self.n_up:] = 1
        self.spin = spin

    # ------------------------------------------------------------------
    # network pieces
    # ------------------------------------------------------------------
    def filter(self, feat, rho, W1, b1, W2, b2, W3, Wenv, sig, cutoff, per_nucleus=False):
        """Gamma(x) = [SiLU(SiLU(x W1 + b1) W2 + b2) W3] * [chi(x_0) W_env],
        chi(x_0) = f_cut(x_0/c) * exp(-sigma_k^2 x_0^2) (Methods, eq. for
        Gamma_m and chi).  With per_nucleus, W1 [M,4,h] and b1 [M,h] differ
        per nucleus (the third-from-last axis of feat)."""
        if per_nucleus:
            z = torch.einsum("bnmk,mkh->bnmh", feat, W1) + b1
        else:
            z = feat @ W1 + b1
        z = silu(z)
        z = silu(z @ W2 + b2)
        radial = fcut(rho / cutoff)[..., None] * torch.exp(-(sig ** 2) * rho[..., None] ** 2)
        return (z @ W3) * (radial @ Wenv)

    def layernorm(self, s):
        mu = s.mean(-1, keepdim=True)
        var = ((s - mu) ** 2).mean(-1, keepdim=True)
        return (s - mu) / torch.sqrt(var + LN_EPS) * self.p["ln_g"] + self.p["ln_b"]

    def embed(self, R):
        """All intermediate embeddings for walkers R [B,n,3]."""
        p, cn, c = self.p, self.model.cutoff_nuc, self.model.cutoff
        B, n = R.shape[0], self.n
        out = {}
        # --- electron-nucleus part: initial embedding h0 (Methods, h^0_i)
        x = R[:, :, None, :] - self.Rn[None, None]                 # [B,n,M,3]
        rho, _ = _safe_norm(x, (x.abs().sum(-1) == 0))
        e = torch.cat([rho[..., None], x], -1)                     # [B,n,M,4]
        ebar = _log1p_over(rho)[..., None] * e
        t = self.nuc_type
        gam = self.filter(e, rho, p["en_W1"][t], p["en_b1"][t], p["en_W2"], p["en_b2"],
                          p["en_W3"], p["en_Wenv"], p["en_sig"], cn, per_nucleus=True)
        val = p["nuc_emb"][t] + ebar @ p["en_Wn"]
        s = (gam * val).sum(2)                                     # [B,n,d]
        y = self.layernorm(s)
        h0 = ((y @ p["glu_Wv"] + p["glu_bv"]) * silu(y @ p["glu_Wg"] + p["glu_bg"])) @ p["glu_Wo"] + p["glu_bo"]
        out["s"], out["h0"] = s, h0
        # --- one message-passing step over electron pairs (Methods, m^alpha_i)
        dr = R[:, :, None, :] - R[:, None, :, :]                   # r_i - r_j  [B,n,n,3]
        eye = torch.eye(n, dtype=torch.bool)[None].expand(B, n, n)
        r, dr_s = _safe_norm(dr, eye)
        ee = torch.cat([r[..., None], dr_s], -1)
        eebar = _log1p_over(r)[..., None] * ee
        same = (self.spin[:, None] == self.spin[None, :])
        m = torch.zeros_like(h0)
        out["m"] = []
        for a in (0, 1):
            mask = (~eye) & (same if a == 0 else ~same)[None]
            gam = self.filter(ee, r, p["ee_W1"][a], p["ee_b1"][a], p["ee_W2"][a], p["ee_b2"][a],
                              p["ee_W3"][a], p["ee_Wenv"][a], p["ee_sig"][a], c)
            pre = (h0 @ p["msg_Wa"][a])[:, :, None, :] + (h0 @ p["msg_Wb"][a])[:, None, :, :] \
                + eebar @ p["msg_We"][a] + p["msg_b"][a]
            ma = (gam * silu(pre) * mask[..., None]).sum(2)
            out["m"].append(ma)
            m = m + ma
        h = h0 + m
        out["h1"] = h
        # --- embedding MLP
        for k in range(self.model.mlp_layers):
            h = silu(h @ p["mlp_W"][k] + p["mlp_b"][k])
        out["h"] = h
        return out

    def envelopes(self, R, spin):
        """phi_l(r_i) = sum_{m,e} pi_{lme} exp(-sigma_me |r_i - R_m|) for the
        electrons of one spin block, all determinants: [B,K,N,N]."""
        p = self.p
        nu = self.n_up
        Rs = R[:, :nu] if spin == 0 else R[:, nu:]
        dist = torch.sqrt(((Rs[:, :, None, :] - self.Rn[None, None]) ** 2).sum(-1))  # [B,N,M]
        basis = torch.exp(-p["env_sigma"][None, None] * dist[..., None])              # [B,N,M,E]
        pi = p["env_pi_up"] if spin == 0 else p["env_pi_dn"]                          # [K,N,M,E]
        return torch.einsum("bime,klme->bkil", basis, pi)

    def orbitals(self, R, h):
        """Phi_{d,sigma}[i,l] = (h_i . W_{d,sigma}[:,l]) * phi_{d,sigma,l}(r_i)."""
        nu = self.n_up
        out = []
        for spin, Wk in ((0, "orb_W_up"), (1, "orb_W_dn")):
            hs = h[:, :nu] if spin == 0 else h[:, nu:]
            proj = torch.einsum("bid,kdl->bkil", hs, self.p[Wk])
            out.append(proj * self.envelopes(R, spin))
        return out

    def log_psi_parts(self, R):
        """Per-determinant (sign, log|det|) and the signed log-sum-exp."""
        h = self.embed(R)["h"]
        phis = self.orbitals(R, h)
        B, K = R.shape[0], self.model.n_det
        sgn = torch.ones(B, K, dtype=DT)
        ld = torch.zeros(B, K, dtype=DT)
        for phi in phis:
            if phi.shape[-1] == 0:
                continue
            s, l = torch.linalg.slogdet(phi)
            sgn = sgn * s
            ld = ld + l
        lmax = ld.max(1, keepdim=True).values
        tot = (sgn * torch.exp(ld - lmax)).sum(1)
        sign = torch.sign(tot)
        logpsi = lmax[:, 0] + torch.log(torch.abs(tot)) + self.jastrow_cusp(R)
        if "jmlp_W1" in self.p:
            lj, sj = self.jastrow_mlp(h)
            logpsi = logpsi + lj
            sign = sign * sj
        if "jatt_q" in self.p:
            la, sa = self.jastrow_att(h)
            logpsi = logpsi + la
            sign = sign * sa
        return sign, logpsi, sgn, ld, phis

    def jastrow_cusp(self, R):
        """log of the cusp Jastrow factor (Methods, global electron
        correlation): the sum over electron pairs i < j of w a^2 / (a + r_ij),
        with (w, a) = (w_par, a_par) for equal spins and (w_anti, a_anti) for
        opposite spins; theta entry jas_cusp = (w_par, a_par, w_anti, a_anti)."""
        R = torch.as_tensor(R, dtype=DT)
        if "jas_cusp" not in self.p or self.n < 2:
            return torch.zeros(R.shape[0], dtype=DT)
        q = self.p["jas_cusp"]
        iu = torch.triu_indices(self.n, self.n, 1)
        rij = torch.linalg.norm(R[:, iu[0]] - R[:, iu[1]], dim=-1)           # [B, pairs]
        nu = self.sys.n_up
        same = (iu[0] < nu) == (iu[1] < nu)
        w = torch.where(same, q[0], q[2])
        a = torch.where(same, q[1], q[3])
        return (w * a * a / (a + rij)).sum(1)

    def jastrow_mlp_terms(self, h):
        """The two per-electron readouts of the MLP Jastrow (Methods, global
        electron correlation): MLP_k(h_i) = w3_k . SiLU(SiLU(h_i W1_k + b1_k)
        W2_k + b2_k) + b3_k for k = 1 (log part) and 2 (node part), over the
        final embeddings h [B,n,d]: returns [B,n,2]."""
        p = self.p
        out = []
        for k in (0, 1):
            z = silu(h @ p["jmlp_W1"][k] + p["jmlp_b1"][k])
            z = silu(z @ p["jmlp_W2"][k] + p["jmlp_b2"][k])
            out.append(z @ p["jmlp_w3"][k] + p["jmlp_b3"][k])
        return torch.stack(out, -1)

    def jastrow_mlp(self, h):
        """(log|J_MLP|, sign J_MLP) with J_MLP = exp(sum_i MLP_1(h_i)) *
        sum_i MLP_2(h_i) (Methods, global electron correlation; the three
        Jastrow terms multiply, their logs add)."""
        t = self.jastrow_mlp_terms(h)
        s1, s2 = t[..., 0].sum(1), t[..., 1].sum(1)
        return s1 + torch.log(torch.abs(s2)), torch.sign(s2)

    def jastrow_att_registers(self, h):
        """Register embeddings of the attention Jastrow (Methods, global
        electron correlation): for register r, the softmax over the electrons
        of the logits h_i . q_r weights the values h_i W^V_r; returns
        V = Concat_r v_r [B, N_reg d_reg]."""
        p = self.p
        logits = torch.einsum("bnd,rd->bnr", h, p["jatt_q"])
        w = torch.softmax(logits, dim=1)                           # over electrons
        vals = torch.einsum("bnd,rde->bnre", h, p["jatt_Wv"])
        v = torch.einsum("bnr,bnre->bre", w, vals)
        return v.reshape(h.shape[0], -1)

    def jastrow_att(self, h):
        """(log|J_att|, sign J_att) with J_att = exp(MLP_1(V)) MLP_2(V) over the
        register embeddings V, each MLP two SiLU hidden layers and a scalar
        linear readout."""
        p = self.p
        V = self.jastrow_att_registers(h)
        out = []
        for k in (0, 1):
            z = silu(V @ p["jatt_W1"][k] + p["jatt_b1"][k])
            z = silu(z @ p["jatt_W2"][k] + p["jatt_b2"][k])
            out.append(z @ p["jatt_w3"][k] + p["jatt_b3"][k])
        return out[0] + torch.log(torch.abs(out[1])), torch.sign(out[1])

    def log_psi(self, R):
        """(sign, log|psi|) for walkers R [B,n,3], psi = exp(J_cusp) J_MLP J_att
        sum_d det Phi_d (J_MLP, J_att = 1 unless the parameters hold their
        weights)."""
        R = torch.as_tensor(R, dtype=DT)
        s, l, *_ = self.log_psi_parts(R)
        return s, l

    # ------------------------------------------------------------------
    # Hamiltonian
    # ------------------------------------------------------------------
    def local_pp(self, r):
        """v_loc,m(r) = -Z_m/r (bare) or -Z_m erf(r/w_m)/r (pseudo-atoms)."""
        w = self.pp_width
        Z = self.Z
        bare = -Z / r
        ws = torch.where(w > 0, w, torch.ones_like(w))
        smooth = -Z * torch.erf(r / ws) / r
        small = r < 1e-10
        lim = -Z * 2.0 / (ws * math.sqrt(math.pi))
        smooth = torch.where(small, lim, smooth)
        return torch.where(w > 0, smooth, bare)

    def potential(self, R):
        """[V_ee, V_en, V_nn] per walker (Methods, Hamiltonian, with the local
        pseudopotential replacing -Z/r on pseudo-atoms)."""
        R = torch.as_tensor(R, dtype=DT)
        B, n = R.shape[:2]
        iu = torch.triu_indices(n, n, 1)
        dr = R[:, iu[0]] - R[:, iu[1]]
        vee = (1.0 / torch.sqrt((dr ** 2).sum(-1))).sum(1)
        rim = torch.sqrt(((R[:, :, None] - self.Rn[None, None]) ** 2).sum(-1))
        ven = self.local_pp(rim).sum((1, 2))
        M = self.Rn.shape[0]
        vnn = 0.0
        for a in range(M):
            for b in range(a + 1, M):
                vnn += float(self.Z[a] * self.Z[b] / torch.linalg.norm(self.Rn[a] - self.Rn[b]))
        return torch.stack([vee, ven, torch.full_like(vee, vnn)], 1)

    def grad_lap(self, R, chunk: int = 64, coords=None):
        """grad log|psi| [B,n,3] and Laplacian of log|psi| [B], by reverse mode
        for the gradient and forward-over-reverse for each diagonal Hessian
        element (exact, no finite differences).  coords (optional) restricts
        the Hessian trace to a subset of the 3n coordinates (timing samples)."""
        from torch.func import grad, jvp, vmap
        R = torch.as_tensor(R, dtype=DT)
        B, n = R.shape[:2]

        def f(x):
            return self.log_psi_parts(x.reshape(1, n, 3))[1][0]

        g_fn = grad(f)
        grads = torch.zeros(B, n * 3, dtype=DT)
        laps = torch.zeros(B, dtype=DT)
        eye = torch.eye(3 * n, dtype=DT)
        if coords is not None:
            eye = eye[torch.as_tensor(coords, dtype=torch.long)]
        for b in range(B):
            x = R[b].reshape(-1).clone()
            grads[b] = g_fn(x)
            tot = 0.0
            for c0 in range(0, eye.shape[0], chunk):
                V = eye[c0:c0 + chunk]
                hv = vmap(lambda v: jvp(g_fn, (x,), (v,))[1])(V)
                tot = tot + (hv * V).sum()
            laps[b] = tot
        return grads.reshape(B, n, 3), laps

    def kinetic(self, R, **kw):
        g, lap = self.grad_lap(R, **kw)
        return -0.5 * (lap + (g ** 2).sum((1, 2)))

    def ecp_nonlocal(self, R, Q=None):
        """Nonlocal pseudopotential: for every electron i and pseudo-atom I with
        |r_i - R_I| < r_max, sum_l v_l(r)(2l+1) (1/N_q) sum_q P_l(cos)
        psi(r_i -> R_I + r Q e_q)/psi, every ratio by full re-evaluation.  The
        rule has N_q points per species (SI, effective core potential:
        tetrahedron 4, octahedron 6, icosahedron 12; default 12)."""
        R = torch.as_tensor(R, dtype=DT)
        B, n = R.shape[:2]
        out = torch.zeros(B, dtype=DT)
        if not self.sys.ecp:
            return out
        nq_of = getattr(self.sys, "ecp_nquad", {}) or {}
        Qs = torch.eye(3, dtype=DT)[None].expand(B, 3, 3) if Q is None else torch.as_tensor(Q, dtype=DT)
        s0, l0 = self.log_psi(R)
        rmax = self.sys.ecp_rmax
        for b in range(B):
            rules = {nq: (Qs[b] @ quadrature_directions(nq).T).T for nq in (4, 6, 12)}   # rotated directions
            jobs = []
            for i in range(n):
                for I in range(self.Rn.shape[0]):
                    sp = int(self.sys.species[I])
                    if sp not in self.sys.ecp:
                        continue
                    v = R[b, i] - self.Rn[I]
                    r = float(torch.linalg.norm(v))
                    if r >= rmax:
                        continue
                    jobs.append((i, I, sp, r, v / r))
            if not jobs:
                continue
            nqs = [int(nq_of.get(sp, 12)) for (_, _, sp, _, _) in jobs]
            first = np.concatenate([[0], np.cumsum(nqs)])
            Rq = R[b][None].repeat(int(first[-1]), 1, 1).clone()
            for k, (i, I, sp, r, u) in enumerate(jobs):
                Rq[first[k]:first[k + 1], i] = self.Rn[I][None] + r * rules[nqs[k]]
            sq, lq = self.log_psi(Rq)
            ratio = (sq * s0[b]) * torch.exp(lq - l0[b])
            tot = 0.0
            for k, (i, I, sp, r, u) in enumerate(jobs):
                cos = rules[nqs[k]] @ u
                rk = ratio[first[k]:first[k + 1]]
                for ch in self.sys.ecp[sp]:
                    vl = float(np.sum(ch.a * np.exp(-ch.alpha * r * r)))
                    Pl = torch.ones_like(cos) if ch.l == 0 else cos
                    tot = tot + vl * (2 * ch.l + 1) * (Pl * rk).mean()
            out[b] = tot
        return out

    def local_energy(self, R, Q=None, **kw):
        """E_L = -1/2 (Lap log|psi| + |grad log|psi||^2) + V_ee + V_en + V_nn + V_NL
        (Methods, local energy).  Returns (E_L [B], parts [B,5])."""
        R = torch.as_tensor(R, dtype=DT)
        kin = self.kinetic(R, **kw)
        V = self.potential(R)
        vnl = self.ecp_nonlocal(R, Q)
        parts = torch.cat([kin[:, None], V, vnl[:, None]], 1)
        return parts.sum(1), parts

    def splus_ratios(self, R, beta):
        """The S+ spin-penalty estimator (SI, low-rank updates in S+
        operator): for the spin-down electron beta and every spin-up electron
        a, psi(pi_{a,beta} r)/psi(r) with the positions of a and beta
        exchanged (a full re-evaluation), and R_beta = 1 - sum_a of them.
        Returns (ratios [B, n_up], R_beta [B])."""
        R = torch.as_tensor(R, dtype=DT)
        s0, l0 = self.log_psi(R)
        out = torch.zeros(R.shape[0], self.n_up, dtype=DT)
        for a in range(self.n_up):
            Rs = R.clone()
            Rs[:, [a, beta]] = R[:, [beta, a]]
            s1, l1 = self.log_psi(Rs)
            out[:, a] = s1 * s0 * torch.exp(l1 - l0)
        return out, 1.0 - out.sum(1)

    # ------------------------------------------------------------------
    # sampling and parameter gradients
    # ------------------------------------------------------------------
    def gmm_log_density(self, r, tau):
        """log rho_global(r) of the global single-electron jump (SI, improved
        Monte Carlo sampling, eq. of rho_global): the charge-weighted mixture
        rho(r) = sum_m Z_m N(r | R_m, tau^2 I) / sum_m Z_m of isotropic
        Gaussians on the nuclei.  r [..., 3]."""
        r = torch.as_tensor(r, dtype=DT)
        d2 = ((r[..., None, :] - self.Rn) ** 2).sum(-1)                 # [..., M]
        log_normal = -d2 / (2.0 * tau * tau) - 1.5 * math.log(2.0 * math.pi * tau * tau)
        return torch.logsumexp(torch.log(self.Z) + log_normal, dim=-1) - torch.log(self.Z.sum())

    def gmm_draw(self, pick, xi, tau):
        """A draw from rho_global from explicit random numbers: component m
        with probability Z_m / sum Z (the first m whose cumulative weight
        exceeds the uniform pick), then R_m + tau xi.  pick [B], xi [B, 3]."""
        pick = torch.as_tensor(pick, dtype=DT)
        xi = torch.as_tensor(xi, dtype=DT)
        cum = torch.cumsum(self.Z, 0) / self.Z.sum()
        m = torch.searchsorted(cum, pick, right=True).clamp(max=self.Rn.shape[0] - 1)
        return self.Rn[m] + tau * xi

    def mcmc_sweep(self, R, step, noise, unif, kinds=None, pick=None, gstep=2.0):
        """Systematic-scan Metropolis over the electrons with a full recompute
        for every proposal (Methods, improved Monte Carlo sampling).  Sweep t
        moves each electron locally, r'_e = r_e + step*xi, accepted iff
        u < (psi'/psi)^2; with kinds[t] == 1 it instead jumps globally to a
        draw of rho_global (gmm_draw, scale gstep), and the acceptance takes
        the factor rho(r_e) / rho(r'_e) of the asymmetric proposal.
        noise [S][n][B][3], unif and pick [S][n][B]."""
        R = torch.as_tensor(R, dtype=DT).clone()
        noise = torch.as_tensor(noise, dtype=DT)
        unif = torch.as_tensor(unif, dtype=DT)
        S = noise.shape[0]
        s, l = self.log_psi(R)
        nacc = torch.zeros(R.shape[0], dtype=torch.long)
        for t in range(S):
            jump = kinds is not None and int(kinds[t]) == 1
            for e in range(self.n):
                Rp = R.clone()
                if jump:
                    Rp[:, e] = self.gmm_draw(pick[t, e], noise[t, e], gstep)
                    log_q = self.gmm_log_density(R[:, e], gstep) - self.gmm_log_density(Rp[:, e], gstep)
                else:
                    Rp[:, e] = R[:, e] + step * noise[t, e]
                    log_q = torch.zeros(R.shape[0], dtype=DT)
                sp, lp = self.log_psi(Rp)
                ratio2 = torch.exp(2.0 * (lp - l) + log_q)
                acc = unif[t, e] < ratio2
                R = torch.where(acc[:, None, None], Rp, R)
                s = torch.where(acc, sp, s)
                l = torch.where(acc, lp, l)
                nacc += acc.long()
        return R, s, l, nacc

    def grad_params(self, R, coeff):
        """sum_w coeff_w d log|psi_w| / d theta, as a dict of arrays."""
        R = torch.as_tensor(R, dtype=DT)
        coeff = torch.as_tensor(coeff, dtype=DT)
        leaves = {k: v.clone().requires_grad_(True) for k, v in self.p.items()}
        saved = self.p
        self.p = leaves
        try:
            _, l = self.log_psi(R)
            tot = (coeff * l).sum()
            grads = torch.autograd.grad(tot, list(leaves.values()), allow_unused=True)
        finally:
            self.p = saved
        return {k: (g if g is not None else torch.zeros_like(leaves[k])).detach()
                for k, g in zip(leaves.keys(), grads)}


def energy_gradient(orc: Oracle, R, e_loc):
    """E[(E_L - mean E_L) grad log|psi|] over the walker batch (Methods,
    energy gradient without the factor 2 of d<E>/d theta)."""
    e = torch.as_tensor(e_loc, dtype=DT)
    W = e.shape[0]
    return orc.grad_params(R, (e - e.mean()) / W)


def per_walker_gradients(orc: Oracle, R, names):
    """O [W][P]: row w is d log|psi_w| / d theta, flattened in the order of
    names (one reverse pass per walker)."""
    R = torch.as_tensor(R, dtype=DT)
    W = R.shape[0]
    rows = []
    for w in range(W):
        c = torch.zeros(W, dtype=DT)
        c[w] = 1.0
        g = orc.grad_params(R, c)
        rows.append(torch.cat([g[k].reshape(-1) for k in names]))
    return torch.stack(rows).numpy()


def spring_step(O, e, lam, eta, delta_prev=None, delta_tilde=None, lam_pinv=None):
    """The natural-gradient update with momentum (Methods, variational Monte
    Carlo, eq. spring): with Obar the walker-centred per-walker gradients
    (rows = walkers) and eps the centred local energies,
      delta = Obar^T (Obar Obar^T + lam I)^-1 (eps - Obar eta delta_prev) + eta delta_prev.
    With an extra gradient delta_tilde (SI, non-hermitian operator gradients
    in Spring, eq. aux_spring), its part in the span of the rows of Obar,
    Obar^T eps~ with eps~ = (Obar Obar^T + lam_pinv I)^-1 Obar delta_tilde (the
    damped pseudo-inverse), joins eps, and the rest is added to delta."""
    O = np.asarray(O, np.float64)
    e = np.asarray(e, np.float64)
    W, P = O.shape
    Ob = O - O.mean(0, keepdims=True)
    eps = e - e.mean()
    dprev = np.zeros(P) if delta_prev is None else np.asarray(delta_prev, np.float64)
    K = Ob @ Ob.T
    rhs = eps - Ob @ (eta * dprev)
    out = eta * dprev
    if delta_tilde is not None:
        dt = np.asarray(delta_tilde, np.float64)
        eps_t = np.linalg.solve(K + lam_pinv * np.eye(W), Ob @ dt)
        rhs = rhs + eps_t
        out = out + dt - Ob.T @ eps_t
    x = np.linalg.solve(K + lam * np.eye(W), rhs)
    return Ob.T @ x + out
