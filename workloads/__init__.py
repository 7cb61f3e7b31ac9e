"""Seeded synthetic workloads for the FiRE hot path.

This module is the only code shared by the FP64 oracle and the HIP path.  It
holds no arithmetic of the method itself: it builds nuclear geometries, spin
assignments, initial walker positions, randomly initialised parameter arrays
(by name and shape), pseudopotential tables, Metropolis noise and quadrature
rotations.  Everything is deterministic given a config id and seed.

The molecules of the paper (S22, acenes, the Fe-S complex) are not
available, so planar hydrocarbons of the same electron counts stand in for
them:

* ``h4``      linear H4 chain (4 electrons, all-electron)
* ``polyene`` zig-zag C12H14, 62 valence electrons
* ``flake``   honeycomb C42H12 flake, 180 valence electrons
* ``uneven``  16 systems (H chains and grown C/H flakes), 20..180 electrons

The cumulene chains H2C=(C=)kCH2 of the runtime-scaling study are built from
standard bond lengths and angles (``cumulene``), not from the paper's
geometry files.

Parameter names and shapes follow the ansatz of the paper's Methods section
("Wave function ansatz"): e-n filters and nuclear embeddings, GLU with
LayerNorm, one message-passing step with separate parallel / antiparallel
weights, an MLP and per-spin orbital projections with exponential envelopes.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence

import numpy as np

BOHR_CC = 2.65      # C-C bond (bohr)
BOHR_CH = 2.06      # C-H bond (bohr)
H_CHAIN_SPACING = 1.8
BASE_SEED = 20250408

# Order of the spawned seed streams (one per consumer).
STREAM_WALKERS, STREAM_WEIGHTS, STREAM_ECP, STREAM_NOISE, STREAM_FD, STREAM_SYSTEMS = range(6)


# ----------------------------------------------------------------------------
# Specifications
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class EcpChannel:
    """One semilocal channel v_l(r) = sum_k a_k exp(-alpha_k r^2)."""
    l: int
    a: np.ndarray       # [n_terms]
    alpha: np.ndarray   # [n_terms]


@dataclasses.dataclass
class System:
    """A molecule: nuclei, charges (effective charges for pseudo-atoms), spins.

    ``nuc_type[m]`` selects the row of the per-nucleus parameter tables
    (embedding vector and first filter layer) used by nucleus m.  It is the
    identity when every nucleus has its own parameters and the species index
    when parameters are shared per element.
    """
    name: str
    R_nuc: np.ndarray          # [M,3] float64
    Z: np.ndarray              # [M] float64 (Z_eff for pseudo-atoms)
    species: np.ndarray        # [M] int32 (0 = H, 1 = C)
    nuc_type: np.ndarray       # [M] int32
    n_up: int
    n_dn: int
    pp_width: np.ndarray       # [M] float64; 0 = bare Coulomb, w>0 -> -Z erf(r/w)/r
    ecp: Dict[int, List[EcpChannel]]  # species -> nonlocal channels
    ecp_rmax: float = 2.0
    # species -> quadrature points of its nonlocal channels (4, 6 or 12;
    # species not named use 12)
    ecp_nquad: Dict[int, int] = dataclasses.field(default_factory=dict)
    elec_atom: Optional[np.ndarray] = None  # [n] atom index used to place electrons

    @property
    def n_el(self) -> int:
        return self.n_up + self.n_dn

    @property
    def n_nuc(self) -> int:
        return int(self.R_nuc.shape[0])


@dataclasses.dataclass
class Model:
    """Hyper-parameters of the finite-range embedding ansatz."""
    width: int = 256
    mlp_layers: int = 2
    n_det: int = 4
    n_env: int = 8
    n_gauss: int = 32
    edge_hidden: Sequence[int] = (16, 8)
    cutoff: float = 5.0
    cutoff_nuc: float = 20.0
    n_nuc_types: int = 0        # rows of per-nucleus tables
    env_sigma_fixed: Optional[float] = None  # C1: a single exp(-|r-R|)
    jas_mlp_width: int = 0      # hidden width of the per-electron MLP Jastrow (0: off)
    jas_att_regs: int = 0       # registers of the attention Jastrow (0: off)
    jas_att_dim: int = 16       # register dimension d_reg
    jas_att_width: int = 0      # hidden width of its readout MLPs


# ----------------------------------------------------------------------------
# Geometries
# ----------------------------------------------------------------------------
def _rot2(v, ang):
    c, s = math.cos(ang), math.sin(ang)
    return np.array([c * v[0] - s * v[1], s * v[0] + c * v[1]])


def h_chain(n_atoms: int, spacing: float = H_CHAIN_SPACING):
    R = np.zeros((n_atoms, 3))
    R[:, 0] = spacing * np.arange(n_atoms)
    return R, np.zeros(n_atoms, np.int32)


def polyene_c12h14(a: float = BOHR_CC, ch: float = BOHR_CH):
    """All-trans zig-zag C12H14 in the xy plane (120 degree angles)."""
    nC = 12
    C = np.array([[k * a * math.cos(math.pi / 6), (k % 2) * a * math.sin(math.pi / 6)]
                  for k in range(nC)])
    H = []
    for k in range(nC):
        nbrs = [j for j in (k - 1, k + 1) if 0 <= j < nC]
        if len(nbrs) == 2:
            u = sum((C[j] - C[k]) / np.linalg.norm(C[j] - C[k]) for j in nbrs)
            H.append(C[k] - ch * u / np.linalg.norm(u))
        else:
            b = (C[nbrs[0]] - C[k]) / a
            for ang in (2 * math.pi / 3, -2 * math.pi / 3):
                H.append(C[k] + ch * _rot2(b, ang))
    R = np.zeros((nC + len(H), 3))
    R[:nC, :2] = C
    R[nC:, :2] = np.array(H)
    species = np.array([1] * nC + [0] * len(H), np.int32)
    return R, species


BOHR_CC_CUMULENE = 2.48   # cumulenic C=C, 1.31 angstrom
BOHR_CH_SP2 = 2.04        # C-H on an sp2 carbon, 1.08 angstrom
HCH_DEG = 118.0           # H-C-H angle of the terminal methylene groups


def cumulene(n_carbon: int, a: float = BOHR_CC_CUMULENE, ch: float = BOHR_CH_SP2,
             hch_deg: float = HCH_DEG):
    """H2C=C=...=CH2 with n_carbon >= 2 carbons on the x axis, then 4 H.

    The chain has n_carbon - 1 cumulated double bonds.  With an odd number of
    them the two methylene groups lie in one plane (xy; ethylene,
    butatriene), with an even number in perpendicular planes (xy and xz;
    allene), as the alternating pi systems of the chain require.  Valence
    electrons with a pseudo-carbon: 4 n_carbon + 4."""
    if n_carbon < 2:
        raise ValueError("a cumulene needs at least two carbons")
    C = np.zeros((n_carbon, 3))
    C[:, 0] = a * np.arange(n_carbon)
    half = math.radians(hch_deg) / 2
    far = C[-1]
    planar = (n_carbon - 1) % 2 == 1
    H = []
    for sgn in (1.0, -1.0):
        H.append(C[0] + ch * np.array([-math.cos(half), sgn * math.sin(half), 0.0]))
    for sgn in (1.0, -1.0):
        side = [0.0, sgn * math.sin(half), 0.0] if planar else [0.0, 0.0, sgn * math.sin(half)]
        H.append(far + ch * np.array([math.cos(half), side[1], side[2]]))
    R = np.concatenate([C, np.array(H)], axis=0)
    species = np.array([1] * n_carbon + [0] * 4, np.int32)
    return R, species


def honeycomb_sites(a: float = BOHR_CC, n_max: int = 400):
    """Honeycomb sites around a hexagon centre, sorted by (radius, angle)."""
    seen, pts = set(), []
    span = int(math.ceil(math.sqrt(n_max))) + 4
    for i in range(-span, span + 1):
        for j in range(-span, span + 1):
            c = np.array([1.5 * a * (i + j), math.sqrt(3) / 2 * a * (i - j)])
            for k in range(6):
                p = c + a * np.array([math.cos(k * math.pi / 3), math.sin(k * math.pi / 3)])
                key = (round(p[0], 6), round(p[1], 6))
                if key not in seen:
                    seen.add(key)
                    pts.append(p)
    pts = np.array(pts)
    r = np.linalg.norm(pts, axis=1)
    ang = np.mod(np.arctan2(pts[:, 1], pts[:, 0]), 2 * math.pi)
    order = np.lexsort((np.round(ang, 9), np.round(r, 9)))
    return pts[order][:n_max]


def _bonds(C, a):
    d = np.linalg.norm(C[:, None] - C[None], axis=-1)
    return (d < 1.01 * a) & (d > 0.1 * a)


def _h_on_carbon(C, k, adj, a, ch):
    nb = np.nonzero(adj[k])[0]
    if len(nb) == 2:
        u = sum((C[j] - C[k]) / a for j in nb)
        return [C[k] - ch * u / np.linalg.norm(u)]
    if len(nb) == 1:
        b = (C[nb[0]] - C[k]) / a
        return [C[k] + ch * _rot2(b, ang) for ang in (2 * math.pi / 3, -2 * math.pi / 3)]
    return []


def flake_c42h12(a: float = BOHR_CC, ch: float = BOHR_CH):
    """42 honeycomb sites nearest a hexagon centre (5 shells, D6h); H on the
    12 two-coordinated carbons of the sqrt(13)*a shell."""
    C = honeycomb_sites(a, 42)
    adj = _bonds(C, a)
    r = np.linalg.norm(C, axis=1)
    H = []
    for k in range(42):
        if abs(r[k] - math.sqrt(13) * a) < 1e-6 and adj[k].sum() == 2:
            H += _h_on_carbon(C, k, adj, a, ch)
    assert len(H) == 12
    R = np.zeros((42 + 12, 3))
    R[:42, :2] = C
    R[42:, :2] = np.array(H)
    return R, np.array([1] * 42 + [0] * 12, np.int32)


def grown_flake(n_el: int, a: float = BOHR_CC, ch: float = BOHR_CH):
    """Connected honeycomb flake with n_el valence electrons (4 per C, 1 per H).

    Sites are added one at a time, always the lowest (radius, angle) site that
    is bonded to the current set.  The carbon count is the smallest k >=
    floor(n_el/5) whose dangling-bond count can host the n_el - 4k hydrogens.
    """
    pool = honeycomb_sites(a, 400)
    adj_all = _bonds(pool, a)
    order = [0]
    inset = np.zeros(len(pool), bool)
    inset[0] = True
    def grow():
        cand = np.nonzero(adj_all[inset].any(0) & ~inset)[0]
        k = int(cand.min())   # pool is sorted by (radius, angle)
        inset[k] = True
        order.append(k)
    k = max(1, n_el // 5)
    while len(order) < k:
        grow()
    while True:
        C = pool[order]
        adj = _bonds(C, a)
        coord = adj.sum(1)
        dangling = int(np.sum(np.where(coord == 2, 1, np.where(coord == 1, 2, 0))))
        nH = n_el - 4 * len(order)
        if nH <= dangling:
            break
        grow()
    assert nH >= 0
    r = np.linalg.norm(C, axis=1)
    ang = np.mod(np.arctan2(C[:, 1], C[:, 0]), 2 * math.pi)
    cand = [k for k in range(len(C)) if coord[k] in (1, 2)]
    cand.sort(key=lambda k: (coord[k], -round(r[k], 9), round(ang[k], 9)))
    H = []
    for k in cand:
        if len(H) >= nH:
            break
        H += _h_on_carbon(C, k, adj, a, ch)[: nH - len(H)]
    R = np.zeros((len(C) + len(H), 3))
    R[:len(C), :2] = C
    if H:
        R[len(C):, :2] = np.array(H)
    return R, np.array([1] * len(C) + [0] * len(H), np.int32)


# ----------------------------------------------------------------------------
# Systems
# ----------------------------------------------------------------------------
def _ecp_tables(rng) -> Dict[int, List[EcpChannel]]:
    """Synthetic semilocal channels l=0,1 for carbon, two Gaussian terms each."""
    chans = []
    for l in (0, 1):
        chans.append(EcpChannel(l=l, a=rng.uniform(-2.0, 2.0, 2), alpha=rng.uniform(0.5, 3.0, 2)))
    return {1: chans}


def make_system(name, R, species, *, pseudo_c=True, nonlocal_ecp=False, ecp_rng=None,
                per_species=False, n_up=None, n_dn=None):
    M = len(species)
    Z = np.where(species == 1, 4.0 if pseudo_c else 6.0, 1.0).astype(np.float64)
    pp_width = np.where((species == 1) & pseudo_c, 0.5, 0.0).astype(np.float64)
    # Electron list: Z_eff electrons per atom in atom order, alternating spins,
    # then a stable reorder so the spin-up electrons come first.
    atoms = np.repeat(np.arange(M), Z.astype(int))
    spins = np.arange(len(atoms)) % 2            # 0 = up, 1 = down
    order = np.argsort(spins, kind="stable")
    elec_atom = atoms[order]
    nu = int((spins == 0).sum()) if n_up is None else n_up
    nd = int((spins == 1).sum()) if n_dn is None else n_dn
    ecp = _ecp_tables(ecp_rng) if nonlocal_ecp else {}
    nuc_type = species.astype(np.int32) if per_species else np.arange(M, dtype=np.int32)
    return System(name=name, R_nuc=np.ascontiguousarray(R, np.float64), Z=Z,
                  species=species.astype(np.int32), nuc_type=nuc_type, n_up=nu, n_dn=nd,
                  pp_width=pp_width, ecp=ecp, elec_atom=elec_atom)


def seeds(config_id: int):
    return np.random.SeedSequence(BASE_SEED + config_id).spawn(6)


# ----------------------------------------------------------------------------
# Parameters
# ----------------------------------------------------------------------------
def param_shapes(system: System, model: Model) -> Dict[str, tuple]:
    """Names and shapes of every parameter array, in canonical order."""
    d, G = model.width, model.n_gauss
    h1, h2 = model.edge_hidden
    T = model.n_nuc_types or system.n_nuc
    M, K, E, L = system.n_nuc, model.n_det, model.n_env, model.mlp_layers
    nu, nd = system.n_up, system.n_dn
    Hj = model.jas_mlp_width
    jm = {} if Hj <= 0 else {
        # per-electron MLP Jastrow: index 0 MLP_1 (log part), 1 MLP_2 (node part)
        "jmlp_W1": (2, d, Hj), "jmlp_b1": (2, Hj), "jmlp_W2": (2, Hj, Hj), "jmlp_b2": (2, Hj),
        "jmlp_w3": (2, Hj), "jmlp_b3": (2,),
    }
    Ra, dr, Ha = model.jas_att_regs, model.jas_att_dim, model.jas_att_width
    ja = {} if Ra <= 0 else {
        # attention Jastrow: queries, value maps, readouts 0 (log part), 1 (node part)
        "jatt_q": (Ra, d), "jatt_Wv": (Ra, d, dr),
        "jatt_W1": (2, Ra * dr, Ha), "jatt_b1": (2, Ha), "jatt_W2": (2, Ha, Ha), "jatt_b2": (2, Ha),
        "jatt_w3": (2, Ha), "jatt_b3": (2,),
    }
    return {
        # electron-nucleus filter Gamma_m and nuclear embeddings
        "en_W1": (T, 4, h1), "en_b1": (T, h1),
        "en_W2": (h1, h2), "en_b2": (h2,),
        "en_W3": (h2, d), "en_Wenv": (G, d), "en_sig": (G,),
        "nuc_emb": (T, d), "en_Wn": (4, d),
        # GLU with LayerNorm
        "ln_g": (d,), "ln_b": (d,),
        "glu_Wv": (d, d), "glu_bv": (d,), "glu_Wg": (d, d), "glu_bg": (d,),
        "glu_Wo": (d, d), "glu_bo": (d,),
        # message passing, alpha = 0 (parallel spins), 1 (antiparallel)
        "msg_Wa": (2, d, d), "msg_Wb": (2, d, d), "msg_We": (2, 4, d), "msg_b": (2, d),
        "ee_W1": (2, 4, h1), "ee_b1": (2, h1), "ee_W2": (2, h1, h2), "ee_b2": (2, h2),
        "ee_W3": (2, h2, d), "ee_Wenv": (2, G, d), "ee_sig": (2, G),
        # embedding MLP
        "mlp_W": (L, d, d), "mlp_b": (L, d),
        # cusp Jastrow (w_par, a_par, w_anti, a_anti)
        "jas_cusp": (4,),
        **jm,
        **ja,
        # orbitals and envelopes
        "orb_W_up": (K, d, nu), "orb_W_dn": (K, d, nd),
        "env_pi_up": (K, nu, M, E), "env_pi_dn": (K, nd, M, E),
        "env_sigma": (M, E),
    }


def init_params(system: System, model: Model, rng) -> Dict[str, np.ndarray]:
    """Matrices N(0, 1/fan_in), biases 0, LayerNorm (1, 0), nuclear
    embeddings N(0,1), envelope weights N(0, 1/(M*N_env)), envelope exponents
    linspace(0.5, 3), Gaussian filter widths (1 + 7k/(G-1))/cutoff; the MLP
    and attention Jastrows' readout vectors N(0, 1/width) and readout biases
    (0, 1); attention queries N(0, 1/d)."""
    shapes = param_shapes(system, model)
    p: Dict[str, np.ndarray] = {}
    G = model.n_gauss
    B = system.n_nuc * model.n_env

    def mat(shape, fan_in):
        return rng.normal(0.0, 1.0 / math.sqrt(fan_in), size=shape)

    for name, shp in shapes.items():
        if name in ("en_sig",):
            p[name] = (1.0 + 7.0 * np.arange(G) / (G - 1)) / model.cutoff_nuc
        elif name == "ee_sig":
            p[name] = np.tile((1.0 + 7.0 * np.arange(G) / (G - 1)) / model.cutoff, (2, 1))
        elif name == "ln_g":
            p[name] = np.ones(shp)
        elif name == "jas_cusp":
            # zero weights by default: J_cusp = 1; (-1/4, a, -1/2, a)
            # gives the electron-electron cusp conditions
            p[name] = np.array([0.0, 1.0, 0.0, 1.0])
        elif name in ("jmlp_w3", "jatt_w3", "jatt_q"):
            p[name] = rng.normal(0.0, 1.0 / math.sqrt(shp[-1]), size=shp)
        elif name in ("jmlp_b3", "jatt_b3"):
            # MLP_1 bias 0; MLP_2 bias 1, so that sum_i MLP_2(h_i) starts near
            # n, away from its zero set
            p[name] = np.array([0.0, 1.0])
        elif name in ("jmlp_b2", "jatt_b2"):
            p[name] = np.zeros(shp)
        elif name == "nuc_emb":
            p[name] = rng.normal(0.0, 1.0, size=shp)
        elif name.startswith("env_pi"):
            p[name] = rng.normal(0.0, 1.0 / math.sqrt(B), size=shp)
        elif name == "env_sigma":
            if model.env_sigma_fixed is not None:
                p[name] = np.full(shp, float(model.env_sigma_fixed))
            else:
                p[name] = np.tile(np.linspace(0.5, 3.0, model.n_env), (system.n_nuc, 1))
        elif len(shp) >= 2 and not name.endswith("_b1") and name not in ("mlp_b", "msg_b", "ee_b2"):
            fan_in = shp[-2]
            p[name] = mat(shp, fan_in)
        else:
            p[name] = np.zeros(shp)
    for k in p:
        p[k] = np.ascontiguousarray(p[k], dtype=np.float64)
        assert p[k].shape == tuple(shapes[k]), (k, p[k].shape, shapes[k])
    return p


def flatten_params(p: Dict[str, np.ndarray], order: Sequence[str]) -> np.ndarray:
    return np.concatenate([p[k].reshape(-1) for k in order]).astype(np.float64)


# ----------------------------------------------------------------------------
# Walkers, noise, rotations, quadrature
# ----------------------------------------------------------------------------
def init_walkers(system: System, W: int, rng, sigma: float = 1.0) -> np.ndarray:
    """Electron k drawn from N(R_atom(k), sigma^2 I)."""
    centre = system.R_nuc[system.elec_atom]       # [n,3]
    return centre[None] + sigma * rng.normal(size=(W, system.n_el, 3))


def mcmc_noise(n_sweeps: int, n_el: int, W: int, rng):
    """Gaussian proposal noise [S][n][W][3] and acceptance uniforms [S][n][W]."""
    xi = rng.normal(size=(n_sweeps, n_el, W, 3))
    u = rng.uniform(size=(n_sweeps, n_el, W))
    return xi, u


def gmm_picks(n_sweeps: int, n_el: int, W: int, rng):
    """Uniforms [S][n][W] that choose the nucleus of each global jump."""
    return rng.uniform(size=(n_sweeps, n_el, W))


def haar_rotations(W: int, rng) -> np.ndarray:
    """Uniformly random rotation matrices [W][3][3] (QR of Gaussian matrices)."""
    A = rng.normal(size=(W, 3, 3))
    Q, Rm = np.linalg.qr(A)
    Q = Q * np.sign(np.diagonal(Rm, axis1=1, axis2=2))[:, None, :]
    det = np.linalg.det(Q)
    Q[det < 0, :, 0] *= -1
    return Q


def icosahedron_vertices() -> np.ndarray:
    """The 12 vertices of a regular icosahedron on the unit sphere: the cyclic
    permutations of (0, +-1, +-phi), normalised."""
    phi = (1 + math.sqrt(5)) / 2
    v = []
    for s1 in (1, -1):
        for s2 in (1, -1):
            v.append((0, s1, s2 * phi))
            v.append((s1, s2 * phi, 0))
            v.append((s2 * phi, 0, s1))
    v = np.array(v, np.float64)
    return v / np.linalg.norm(v, axis=1, keepdims=True)


# ----------------------------------------------------------------------------
# The configurations
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class Workload:
    config_id: int
    name: str
    systems: List[System]
    model: Model
    walkers: int
    precision: str
    params: List[Dict[str, np.ndarray]]
    R: List[np.ndarray]
    step: float = 0.2
    sweeps: int = 10
    refresh_every: int = 50
    seeds: Optional[list] = None


def make_model(system: System, **kw) -> Model:
    m = Model(**kw)
    if m.n_nuc_types == 0:
        m.n_nuc_types = int(system.nuc_type.max()) + 1
    return m


def config(config_id: int, walkers: Optional[int] = None, seed_offset: int = 0) -> Workload:
    """Config 0: H4 FP64; 1: C12H14 FP32; 2: C12H14 gradient; 3: C42H12 180 e-
    BF16-hybrid with nonlocal ECP; 4: 16 uneven systems."""
    ss = np.random.SeedSequence(BASE_SEED + config_id + 1 + seed_offset).spawn(6)
    rw = np.random.default_rng(ss[STREAM_WALKERS])
    rp = np.random.default_rng(ss[STREAM_WEIGHTS])
    re = np.random.default_rng(ss[STREAM_ECP])
    if config_id == 0:
        R, sp = h_chain(4)
        s = make_system("H4", R, sp, pseudo_c=False)
        m = make_model(s, width=32, mlp_layers=1, n_det=1, n_env=1, cutoff=5.0,
                       cutoff_nuc=20.0, env_sigma_fixed=1.0)
        W, prec, sweeps = 64, "fp64", 10
    elif config_id in (1, 2):
        R, sp = polyene_c12h14()
        s = make_system("C12H14", R, sp, pseudo_c=True)
        m = make_model(s, width=256, mlp_layers=2, n_det=4, n_env=8, cutoff=5.0, cutoff_nuc=20.0)
        W = 1024 if config_id == 1 else 4096
        prec, sweeps = "fp32", 100
    elif config_id == 3:
        R, sp = flake_c42h12()
        s = make_system("C42H12", R, sp, pseudo_c=True, nonlocal_ecp=True, ecp_rng=re)
        m = make_model(s, width=256, mlp_layers=3, n_det=16, n_env=8, cutoff=5.0, cutoff_nuc=20.0)
        W, prec, sweeps = 4096, "bf16", 10
    elif config_id == 4:
        rs = np.random.default_rng(ss[STREAM_SYSTEMS])
        systems = []
        for k in range(16):
            n = int(rs.integers(20, 181))
            if rs.uniform() < 0.5:
                R, sp = h_chain(n)
            else:
                R, sp = grown_flake(n)
            sk = make_system(f"S{k}_n{n}", R, sp, pseudo_c=True, per_species=True)
            # the uneven batch names no nonlocal channels: local pseudopotential on C only
            sk.ecp = {}
            systems.append(sk)
        m = Model(width=256, mlp_layers=3, n_det=4, n_env=8, cutoff=5.0, cutoff_nuc=20.0,
                  n_nuc_types=2)
        W = 512
        params = [init_params(sk, m, rp) for sk in systems]
        Rs = [init_walkers(sk, walkers or W, rw) for sk in systems]
        return Workload(4, "uneven16", systems, m, walkers or W, "bf16", params, Rs,
                        sweeps=1, seeds=ss)
    else:
        raise ValueError(config_id)
    W = walkers or W
    params = init_params(s, m, rp)
    R0 = init_walkers(s, W, rw)
    return Workload(config_id, s.name, [s], m, W, prec, [params], [R0], sweeps=sweeps, seeds=ss)


def noise_for(work: Workload, n_sweeps: int, W: Optional[int] = None, system: int = 0):
    rn = np.random.default_rng(work.seeds[STREAM_NOISE].spawn(system + 1)[system])
    return mcmc_noise(n_sweeps, work.systems[system].n_el, W or work.walkers, rn)


def fd_directions(work: Workload, n_dir: int = 32, skip=("jas_cusp",)):
    """Seeded unit directions in parameter space, zero on the entries named
    in skip (drawn over the remaining entries only)."""
    rf = np.random.default_rng(work.seeds[STREAM_FD])
    shapes = param_shapes(work.systems[0], work.model)
    sizes = [(k, int(np.prod(s))) for k, s in shapes.items()]
    P = sum(n for _, n in sizes)
    keep = np.ones(P, bool)
    o = 0
    for k, n in sizes:
        if k in skip:
            keep[o:o + n] = False
        o += n
    v = np.zeros((n_dir, P))
    v[:, keep] = rf.normal(size=(n_dir, int(keep.sum())))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def hydrogen_atom(W: int = 16, seed: int = 0):
    """One electron, one proton at the origin, with the network parameters
    set so that h_i is a constant vector and Phi = const * exp(-r): the
    exact ground state, local energy -1/2 hartree everywhere."""
    R = np.zeros((1, 3))
    s = make_system("H", R, np.zeros(1, np.int32), pseudo_c=False, n_up=1, n_dn=0)
    m = make_model(s, width=8, mlp_layers=1, n_det=1, n_env=1, cutoff=5.0, cutoff_nuc=20.0,
                   env_sigma_fixed=1.0)
    rng = np.random.default_rng(seed)
    p = init_params(s, m, rng)
    zero_network(p)
    p["orb_W_up"][:] = 1.0 / m.width
    p["env_pi_up"][:] = 1.0
    walk = rng.normal(size=(W, 1, 3))
    return s, m, p, walk


def zero_network(p: Dict[str, np.ndarray]):
    """Every embedding-network weight matrix and bias to zero except the last
    MLP bias (set to one), so that h_i = SiLU(1) in every channel."""
    for k in p:
        if k.startswith(("en_W", "en_b", "glu_", "msg_", "ee_W", "ee_b", "mlp_", "nuc_emb")):
            p[k][:] = 0.0
    p["ln_g"][:] = 1.0
    p["ln_b"][:] = 0.0
    p["mlp_b"][-1][:] = 1.0


# entries of theta that belong to one molecule (orbital weights and
# envelopes); every entry before them is shared by an uneven batch
PRIVATE_NAMES = ("orb_W_up", "orb_W_dn", "env_pi_up", "env_pi_dn", "env_sigma")


def batch_params(params_list):
    """(shared, private) for an uneven batch: the shared entries are taken
    from the first system's parameters, the private ones from each system."""
    shared = {k: v for k, v in params_list[0].items() if k not in PRIVATE_NAMES}
    private = [{k: p[k] for k in PRIVATE_NAMES} for p in params_list]
    return shared, private


def system_params(shared, private_k):
    """One system's full parameter set inside an uneven batch."""
    out = dict(shared)
    out.update(private_k)
    return out
