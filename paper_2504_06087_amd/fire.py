"""Thin ctypes binding of libfire (argument marshalling only).

Every step of the hot path runs in the HIP kernels of libfire.so; PyTorch
supplies device memory and the current stream.  Importing this module fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfire.so")

FIRE_FP64, FIRE_FP32, FIRE_BF16_HYBRID = 0, 1, 2
PRECISIONS = {"fp64": FIRE_FP64, "fp32": FIRE_FP32, "bf16": FIRE_BF16_HYBRID}
W_NBR_OVERFLOW, W_UPD_OVERFLOW, W_SINGULAR, W_NONFINITE, W_DETSUM_ZERO = 1, 2, 4, 8, 16

EXPORTS = ["fire_create", "fire_destroy", "fire_param_layout", "fire_num_params", "fire_sizes",
           "fire_state_layout", "fire_set_params", "fire_set_overlap", "fire_set_ecp_chunk", "fire_eval_logpsi", "fire_eval_logpsi_noalloc",
           "fire_mcmc_sweep", "fire_mcmc_sweep_mixed", "fire_adapt_step",
           "fire_local_energy", "fire_ecp_nonlocal", "fire_grad_params", "fire_spring_step", "fire_splus_ratios", "fire_sync_status",
           "fire_profile_begin", "fire_profile_end", "fire_status_string",
           "fire_batch_create", "fire_batch_destroy", "fire_batch_num_params", "fire_batch_system",
           "fire_batch_sizes", "fire_batch_set_params", "fire_batch_step", "fire_batch_graph_create",
           "fire_graph_launch", "fire_graph_destroy", "fire_autotune", "fire_autotune_count",
           "fire_autotune_clear", "fire_autotune_save", "fire_autotune_load"]


class FireEcpChannel(ctypes.Structure):
    _fields_ = [("species", ctypes.c_int), ("l", ctypes.c_int), ("n_terms", ctypes.c_int),
                ("a", ctypes.POINTER(ctypes.c_double)), ("alpha", ctypes.POINTER(ctypes.c_double)),
                ("n_quad", ctypes.c_int)]


class FireSystemDesc(ctypes.Structure):
    _fields_ = [("n_nuc", ctypes.c_int), ("R_nuc", ctypes.POINTER(ctypes.c_double)),
                ("Z", ctypes.POINTER(ctypes.c_double)), ("species", ctypes.POINTER(ctypes.c_int)),
                ("nuc_type", ctypes.POINTER(ctypes.c_int)), ("pp_width", ctypes.POINTER(ctypes.c_double)),
                ("n_up", ctypes.c_int), ("n_dn", ctypes.c_int), ("n_ecp", ctypes.c_int),
                ("ecp", ctypes.POINTER(FireEcpChannel)), ("ecp_rmax", ctypes.c_double)]


class FireModelDesc(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int), ("mlp_layers", ctypes.c_int), ("n_det", ctypes.c_int),
                ("n_env", ctypes.c_int), ("n_gauss", ctypes.c_int), ("edge_h1", ctypes.c_int),
                ("edge_h2", ctypes.c_int), ("n_nuc_types", ctypes.c_int), ("cutoff", ctypes.c_double),
                ("cutoff_nuc", ctypes.c_double), ("precision", ctypes.c_int), ("max_walkers", ctypes.c_int),
                ("cap_nbr", ctypes.c_int), ("cap_upd", ctypes.c_int), ("refresh_every", ctypes.c_int),
                ("bf16_split", ctypes.c_int), ("jas_mlp_width", ctypes.c_int), ("jas_att_regs", ctypes.c_int),
                ("jas_att_dim", ctypes.c_int), ("jas_att_width", ctypes.c_int)]


class FireParamEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("offset", ctypes.c_int64), ("ndim", ctypes.c_int32),
                ("shape", ctypes.c_int32 * 4)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libfire.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libfire.so not built at {LIB_PATH}; run paper_2504_06087_amd/build.py")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_void_p
    st = ctypes.c_int32
    lib.fire_create.argtypes = [ctypes.POINTER(FireSystemDesc), ctypes.POINTER(FireModelDesc), ctypes.POINTER(P)]
    lib.fire_destroy.argtypes = [P]
    lib.fire_param_layout.argtypes = [P, ctypes.POINTER(FireParamEntry), ctypes.POINTER(I)]
    lib.fire_num_params.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.fire_sizes.argtypes = [P, I, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t),
                               ctypes.POINTER(ctypes.c_size_t)]
    lib.fire_state_layout.argtypes = [P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.fire_set_params.argtypes = [P, V, V, V]
    lib.fire_set_overlap.argtypes = [P, I]
    lib.fire_set_ecp_chunk.argtypes = [P, I]
    lib.fire_eval_logpsi.argtypes = [P, I, V, V, V, V, V, V, V]
    lib.fire_eval_logpsi_noalloc.argtypes = [P, I, V, V, V, V, V, V]
    lib.fire_mcmc_sweep.argtypes = [P, I, V, V, V, I, D, V, V, ctypes.c_uint64, ctypes.c_uint64, V, V, V, V, V]
    lib.fire_adapt_step.argtypes = [D, ctypes.c_int64, ctypes.c_int64, D, D, ctypes.POINTER(ctypes.c_double)]
    lib.fire_mcmc_sweep_mixed.argtypes = [P, I, V, V, V, I, D, D, ctypes.POINTER(ctypes.c_int32), V, V, V, V, V, V,
                                          V, V]
    lib.fire_local_energy.argtypes = [P, I, V, V, V, V, V, V, V, V, V]
    lib.fire_ecp_nonlocal.argtypes = [P, I, V, V, V, V, V, V, V]
    lib.fire_grad_params.argtypes = [P, I, V, V, V, V, V, V, V, V]
    lib.fire_spring_step.argtypes = [P, I, V, V, D, D, V, V, D, V, V, V, V]
    lib.fire_splus_ratios.argtypes = [P, I, V, V, V, I, V, V, V, V]
    lib.fire_sync_status.argtypes = [P, V, V, I, ctypes.POINTER(ctypes.c_int32)]
    lib.fire_profile_begin.argtypes = [P, V, V, I]
    lib.fire_profile_end.argtypes = [P, V, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.fire_batch_create.argtypes = [ctypes.POINTER(FireSystemDesc), I, ctypes.POINTER(FireModelDesc),
                                      ctypes.POINTER(P)]
    lib.fire_batch_destroy.argtypes = [P]
    lib.fire_batch_num_params.argtypes = [P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
    lib.fire_batch_system.argtypes = [P, I, ctypes.POINTER(P), ctypes.POINTER(ctypes.c_int64)]
    lib.fire_batch_sizes.argtypes = [P, ctypes.POINTER(ctypes.c_int), I, ctypes.POINTER(ctypes.c_size_t),
                                     ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]
    lib.fire_batch_set_params.argtypes = [P, V, V, V]
    lib.fire_batch_step.argtypes = [P, ctypes.POINTER(ctypes.c_int), V, V, V, I, D, V, V, V, V, V, V, V]
    lib.fire_batch_graph_create.argtypes = [P, ctypes.POINTER(ctypes.c_int), V, V, V, I, D, V, V, V, V, V, V,
                                            ctypes.POINTER(P)]
    lib.fire_graph_launch.argtypes = [P, V]
    lib.fire_graph_destroy.argtypes = [P]
    lib.fire_autotune.argtypes = [I]
    lib.fire_autotune_count.argtypes = [ctypes.POINTER(ctypes.c_int)]
    lib.fire_autotune_clear.argtypes = []
    lib.fire_autotune_save.argtypes = [ctypes.c_char_p]
    lib.fire_autotune_load.argtypes = [ctypes.c_char_p]
    lib.fire_status_string.argtypes = [st]
    lib.fire_status_string.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "fire_status_string":
            getattr(lib, name).restype = st
    _lib = lib
    return lib


class FireError(RuntimeError):
    pass


def adapt_step(step: float, accepted: int, proposed: int, target: float = 0.5, gain: float = 1.0) -> float:
    """New local-move scale from the acceptance of the last sweeps
    (fire_adapt_step)."""
    out = ctypes.c_double()
    _check(load().fire_adapt_step(float(step), int(accepted), int(proposed), float(target), float(gain),
                                  ctypes.byref(out)), "fire_adapt_step")
    return out.value


def _check(code: int, what: str):
    if code != 0:
        raise FireError(f"{what}: {load().fire_status_string(code).decode()} ({code})")


def _dp(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _f64(x, dev):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev).contiguous()


def _system_desc(system, keep: list) -> FireSystemDesc:
    """The C descriptor of a molecule; host arrays it points to go in keep."""
    h = dict(R=np.ascontiguousarray(system.R_nuc, np.float64).reshape(-1),
             Z=np.ascontiguousarray(system.Z, np.float64), sp=np.ascontiguousarray(system.species, np.int32),
             nt=np.ascontiguousarray(system.nuc_type, np.int32),
             pw=np.ascontiguousarray(system.pp_width, np.float64))
    keep.append(h)
    chans = []
    for sp, lst in system.ecp.items():
        for ch in lst:
            a = np.ascontiguousarray(ch.a, np.float64)
            al = np.ascontiguousarray(ch.alpha, np.float64)
            keep += [a, al]
            nq = int(getattr(system, "ecp_nquad", {}).get(sp, 12))
            chans.append(FireEcpChannel(int(sp), int(ch.l), len(a),
                                        a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                        al.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), nq))
    arr = (FireEcpChannel * max(1, len(chans)))(*chans)
    keep.append(arr)
    dp = lambda a, t: a.ctypes.data_as(ctypes.POINTER(t))
    return FireSystemDesc(system.n_nuc, dp(h["R"], ctypes.c_double), dp(h["Z"], ctypes.c_double),
                          dp(h["sp"], ctypes.c_int), dp(h["nt"], ctypes.c_int), dp(h["pw"], ctypes.c_double),
                          system.n_up, system.n_dn, len(chans), arr, float(system.ecp_rmax))


def _param_layout(h):
    lib = load()
    cnt = ctypes.c_int(0)
    _check(lib.fire_param_layout(h, None, ctypes.byref(cnt)), "fire_param_layout")
    ents = (FireParamEntry * cnt.value)()
    _check(lib.fire_param_layout(h, ents, ctypes.byref(cnt)), "fire_param_layout")
    return [(e.name.decode(), int(e.offset), tuple(e.shape[:e.ndim])) for e in ents]


def _jastrow_fields(model):
    """(jas_mlp_width, jas_att_regs, jas_att_dim, jas_att_width) of a model."""
    regs = int(getattr(model, "jas_att_regs", 0))
    return (int(getattr(model, "jas_mlp_width", 0)), regs, int(getattr(model, "jas_att_dim", 0)) if regs else 0,
            int(getattr(model, "jas_att_width", 0)) if regs else 0)


class Fire:
    """One handle of libfire for one molecule and one parameter set."""

    def __init__(self, system, model, precision: str = "fp64", max_walkers: int = 1024,
                 cap_nbr: Optional[int] = None, cap_upd: Optional[int] = None, refresh_every: int = 50,
                 device: str = "cuda", bf16_split: int = 0):
        lib = load()
        self.system, self.model, self.precision = system, model, precision
        self.device = torch.device(device)
        n = system.n_el
        self.n = n
        self._keep = []
        sd = _system_desc(system, self._keep)
        cap_nbr = cap_nbr if cap_nbr is not None else min(n - 1, 64) if n > 1 else 1
        cap_upd = cap_upd if cap_upd is not None else min(n, 96)
        self.cap_nbr, self.cap_upd = max(1, cap_nbr), max(1, cap_upd)
        md = FireModelDesc(model.width, model.mlp_layers, model.n_det, model.n_env, model.n_gauss,
                           int(model.edge_hidden[0]), int(model.edge_hidden[1]), int(model.n_nuc_types),
                           float(model.cutoff), float(model.cutoff_nuc), PRECISIONS[precision], int(max_walkers),
                           self.cap_nbr, self.cap_upd, int(refresh_every), int(bf16_split),
                           *_jastrow_fields(model))
        self.max_walkers = max_walkers
        hd = ctypes.c_void_p()
        _check(lib.fire_create(ctypes.byref(sd), ctypes.byref(md), ctypes.byref(hd)), "fire_create")
        self.h = hd
        self.layout = _param_layout(self.h)
        P = ctypes.c_int64(0)
        _check(lib.fire_num_params(self.h, ctypes.byref(P)), "fire_num_params")
        self.P = int(P.value)
        offs = (ctypes.c_size_t * 11)()
        stride = ctypes.c_size_t(0)
        _check(lib.fire_state_layout(self.h, offs, ctypes.byref(stride)), "fire_state_layout")
        self.state_offsets = list(offs)
        self.state_stride = int(stride.value)
        self.params_buf = None
        self.theta = None
        # counters that FireLogPsi uses to see whether the parameters or a
        # state buffer changed between its forward and backward
        self.params_version = 0
        self._state_versions = {}

    def __del__(self):
        try:
            if getattr(self, "h", None) is not None and _lib is not None:
                _lib.fire_destroy(self.h)
        except Exception:
            pass

    # ------------------------------------------------------------------
    def flatten(self, params: Dict[str, np.ndarray]) -> np.ndarray:
        """theta in the library's layout from named arrays (shapes checked)."""
        out = np.zeros(self.P, np.float64)
        for name, off, shape in self.layout:
            a = np.asarray(params[name], np.float64)
            if tuple(a.shape) != tuple(shape):
                raise ValueError(f"{name}: shape {a.shape} != {shape}")
            out[off:off + a.size] = a.reshape(-1)
        return out

    def unflatten(self, theta) -> Dict[str, np.ndarray]:
        t = np.asarray(theta)
        return {name: t[off:off + int(np.prod(shape))].reshape(shape) for name, off, shape in self.layout}

    def sizes(self, W: int):
        p, s, w = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().fire_sizes(self.h, int(W), ctypes.byref(p), ctypes.byref(s), ctypes.byref(w)), "fire_sizes")
        return p.value, s.value, w.value

    def set_overlap(self, on: bool):
        """Stream overlap inside local_energy (fire_set_overlap; off by default)."""
        _check(load().fire_set_overlap(self.h, int(bool(on))), "fire_set_overlap")

    def set_ecp_chunk(self, max_jobs: int):
        """Cap on the pseudopotential quadrature jobs per chunk (fire_set_ecp_chunk;
        0 = automatic).  Call sizes()/buffers() afterwards."""
        _check(load().fire_set_ecp_chunk(self.h, int(max_jobs)), "fire_set_ecp_chunk")

    def set_params(self, params):
        theta = params if isinstance(params, torch.Tensor) else _f64(self.flatten(params), self.device)
        pb, _, _ = self.sizes(1)
        self.params_buf = torch.empty(pb, dtype=torch.uint8, device=self.device)
        self.theta = theta
        _check(load().fire_set_params(self.h, _dp(theta), _dp(self.params_buf), _stream()), "fire_set_params")
        self.params_version += 1

    def buffers(self, W: int):
        _, s, w = self.sizes(W)
        return (torch.empty(s, dtype=torch.uint8, device=self.device),
                torch.empty(w, dtype=torch.uint8, device=self.device))

    # ------------------------------------------------------------------
    def state_version(self, state) -> int:
        return self._state_versions.get(state.data_ptr(), 0)

    def _touch(self, state):
        k = state.data_ptr()
        self._state_versions[k] = self._state_versions.get(k, 0) + 1

    def eval_logpsi(self, R, state, ws):
        W = R.shape[0]
        sign = torch.empty(W, dtype=torch.float64, device=self.device)
        logpsi = torch.empty_like(sign)
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        _check(load().fire_eval_logpsi(self.h, W, _dp(R), _dp(state), _dp(ws), _dp(sign), _dp(logpsi),
                                       _dp(status), _stream()), "fire_eval_logpsi")
        self._touch(state)
        return sign, logpsi, status

    def eval_logpsi_noalloc(self, R, state):
        """fire_eval_logpsi_noalloc: the evaluation with the library's own
        per-GPU scratch array as workspace (allocation-free)."""
        W = R.shape[0]
        sign = torch.empty(W, dtype=torch.float64, device=self.device)
        logpsi = torch.empty_like(sign)
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        _check(load().fire_eval_logpsi_noalloc(self.h, W, _dp(R), _dp(state), _dp(sign), _dp(logpsi), _dp(status),
                                               _stream()), "fire_eval_logpsi_noalloc")
        self._touch(state)
        return sign, logpsi, status

    def mcmc_sweep(self, R, state, ws, n_sweeps, step, noise=None, unif=None, n_accept=None, seed: int = 0,
                   counter: int = 0):
        """Metropolis sweeps; with noise and unif None the library draws the
        random numbers itself (Philox4x32-10, key seed, counter base counter)."""
        W = R.shape[0]
        if n_accept is None:
            n_accept = torch.zeros(W, dtype=torch.int32, device=self.device)
        sign = torch.empty(W, dtype=torch.float64, device=self.device)
        logpsi = torch.empty_like(sign)
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        _check(load().fire_mcmc_sweep(self.h, W, _dp(R), _dp(state), _dp(ws), int(n_sweeps), float(step),
                                      _dp(noise), _dp(unif), int(seed), int(counter), _dp(n_accept), _dp(logpsi),
                                      _dp(sign), _dp(status), _stream()), "fire_mcmc_sweep")
        self._touch(state)
        return n_accept, sign, logpsi, status

    def mcmc_sweep_mixed(self, R, state, ws, kinds, step, global_step, noise, unif, pick, n_accept=None):
        """Sweeps of local moves (kinds[t] = 0) and global single-electron
        jumps (kinds[t] = 1); pick [S][n][W] uniforms (None if no sweep is
        global)."""
        W = R.shape[0]
        if n_accept is None:
            n_accept = torch.zeros(W, dtype=torch.int32, device=self.device)
        sign = torch.empty(W, dtype=torch.float64, device=self.device)
        logpsi = torch.empty_like(sign)
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        k = (ctypes.c_int32 * len(kinds))(*[int(x) for x in kinds])
        _check(load().fire_mcmc_sweep_mixed(self.h, W, _dp(R), _dp(state), _dp(ws), len(kinds), float(step),
                                            float(global_step), k, _dp(noise), _dp(unif), _dp(pick),
                                            _dp(n_accept), _dp(logpsi), _dp(sign), _dp(status), _stream()),
               "fire_mcmc_sweep_mixed")
        self._touch(state)
        return n_accept, sign, logpsi, status

    def local_energy(self, R, state, ws, quad_rot=None, want_grad=False):
        W = R.shape[0]
        e = torch.empty(W, dtype=torch.float64, device=self.device)
        parts = torch.empty(W, 5, dtype=torch.float64, device=self.device)
        g = torch.empty(W, self.n, 3, dtype=torch.float64, device=self.device) if want_grad else None
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        _check(load().fire_local_energy(self.h, W, _dp(R), _dp(state), _dp(ws), _dp(quad_rot), _dp(e), _dp(parts),
                                        _dp(g), _dp(status), _stream()), "fire_local_energy")
        return e, parts, g, status

    def ecp_nonlocal(self, R, state, ws, quad_rot=None):
        W = R.shape[0]
        v = torch.empty(W, dtype=torch.float64, device=self.device)
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        _check(load().fire_ecp_nonlocal(self.h, W, _dp(R), _dp(state), _dp(ws), _dp(quad_rot), _dp(v),
                                        _dp(status), _stream()), "fire_ecp_nonlocal")
        return v, status

    def grad_params(self, R, state, ws, coeff, per_walker=None):
        """sum_w coeff_w d log|psi_w|/d theta; with per_walker (a [W][P] FP64
        tensor) also every walker's gradient."""
        W = R.shape[0]
        g = torch.empty(self.P, dtype=torch.float64, device=self.device)
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        _check(load().fire_grad_params(self.h, W, _dp(R), _dp(state), _dp(ws), _dp(coeff), _dp(g), _dp(per_walker),
                                       _dp(status), _stream()), "fire_grad_params")
        return g, status

    def splus_ratios(self, R, state, ws, beta: int):
        """fire_splus_ratios: psi(pi_{a,beta} r)/psi(r) for every spin-up a,
        and R_beta = 1 - sum_a; returns (ratios [W][n_up], r_beta [W], status)."""
        W = R.shape[0]
        ratios = torch.empty(W, self.system.n_up, dtype=torch.float64, device=self.device)
        rb = torch.empty(W, dtype=torch.float64, device=self.device)
        status = torch.empty(W, dtype=torch.int32, device=self.device)
        _check(load().fire_splus_ratios(self.h, W, _dp(R), _dp(state), _dp(ws), int(beta), _dp(ratios), _dp(rb),
                                        _dp(status), _stream()), "fire_splus_ratios")
        return ratios, rb, status

    def spring_step(self, O, e_loc, ws, lam, eta, delta_prev=None, delta_tilde=None, lam_pinv=0.0):
        """fire_spring_step: the natural-gradient update from per-walker
        gradients O [W][P] and local energies; returns (delta [P], info)."""
        W = O.shape[0]
        delta = torch.empty(self.P, dtype=torch.float64, device=self.device)
        info = torch.empty(1, dtype=torch.int32, device=self.device)
        _check(load().fire_spring_step(self.h, W, _dp(O), _dp(e_loc), float(lam), float(eta), _dp(delta_prev),
                                       _dp(delta_tilde), float(lam_pinv), _dp(delta), _dp(ws), _dp(info), _stream()),
               "fire_spring_step")
        return delta, info

    def profile_begin(self, capacity: int = 200000):
        self._prof_counters = torch.zeros(capacity, dtype=torch.int32, device=self.device)
        _check(load().fire_profile_begin(self.h, _stream(), _dp(self._prof_counters), capacity), "fire_profile_begin")

    def profile_end(self):
        """{kind: (launches, ms, flops, bytes)} for the GEMM kinds f64, f32, bf16, bf16x3."""
        la = (ctypes.c_int64 * 4)()
        ms = (ctypes.c_double * 4)()
        fl = (ctypes.c_double * 4)()
        by = (ctypes.c_double * 4)()
        _check(load().fire_profile_end(self.h, _stream(), la, ms, fl, by), "fire_profile_end")
        names = ["f64", "f32", "bf16", "bf16x3"]
        return {names[k]: (int(la[k]), float(ms[k]), float(fl[k]), float(by[k])) for k in range(4) if la[k]}

    # ------------------------------------------------------------------
    def state_view(self, state, W, which: str):
        """A typed view of one cached array for all W walkers (debug/tests)."""
        names = ["h0", "proj", "m", "phi", "env", "inv", "dsign", "dlog", "lpsi", "spsi", "jas"]
        k = names.index(which)
        tsz = 8 if self.precision == "fp64" else 4
        isz = 4 if self.precision == "fp32" else 8
        n, d, K = self.n, self.model.width, self.model.n_det
        ppd = self.system.n_up ** 2 + self.system.n_dn ** 2
        count = {"h0": n * d, "proj": n * 4 * d, "m": n * d, "phi": K * ppd, "env": K * ppd, "inv": K * ppd,
                 "dsign": 2 * K, "dlog": 2 * K, "lpsi": 1, "spsi": 1, "jas": 1}[which]
        esz = {"inv": isz, "dsign": 8, "dlog": 8, "lpsi": 8, "spsi": 8, "jas": 8}.get(which, tsz)
        dt = torch.float64 if esz == 8 else torch.float32
        rec = state[:W * self.state_stride].view(W, self.state_stride)
        off = self.state_offsets[k]
        return rec[:, off:off + count * esz].contiguous().view(dt)


PRIVATE_NAMES = ("orb_W_up", "orb_W_dn", "env_pi_up", "env_pi_dn", "env_sigma")


class FireBatch:
    """Several molecules of uneven electron counts under one model: shared
    embedding parameters, per-system orbitals and envelopes.  A step runs
    evaluation, sweeps, local energy and the parameter gradient for every
    system; it can be captured once into a HIP graph and replayed."""

    def __init__(self, systems, model, precision: str = "bf16", walkers=(512,), cap_nbr: int = 48,
                 cap_upd: int = 64, refresh_every: int = 50, bf16_split: int = 0, device: str = "cuda"):
        lib = load()
        self.systems, self.model, self.precision = list(systems), model, precision
        self.device = torch.device(device)
        self.W = [int(w) for w in walkers]
        if len(self.W) != len(self.systems):
            raise ValueError("one walker count per system")
        self.n = [s.n_el for s in self.systems]
        self._keep = []
        descs = (FireSystemDesc * len(self.systems))(*[_system_desc(s, self._keep) for s in self.systems])
        self._keep.append(descs)
        md = FireModelDesc(model.width, model.mlp_layers, model.n_det, model.n_env, model.n_gauss,
                           int(model.edge_hidden[0]), int(model.edge_hidden[1]), int(model.n_nuc_types),
                           float(model.cutoff), float(model.cutoff_nuc), PRECISIONS[precision], max(self.W),
                           int(cap_nbr), int(cap_upd), int(refresh_every), int(bf16_split),
                           *_jastrow_fields(model))
        b = ctypes.c_void_p()
        _check(lib.fire_batch_create(descs, len(self.systems), ctypes.byref(md), ctypes.byref(b)),
               "fire_batch_create")
        self.b = b
        pt, ps = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.fire_batch_num_params(self.b, ctypes.byref(pt), ctypes.byref(ps)), "fire_batch_num_params")
        self.P, self.P_shared = int(pt.value), int(ps.value)
        self.handles, self.priv_off, self.layouts = [], [], []
        for k in range(len(self.systems)):
            h, o = ctypes.c_void_p(), ctypes.c_int64()
            _check(lib.fire_batch_system(self.b, k, ctypes.byref(h), ctypes.byref(o)), "fire_batch_system")
            self.handles.append(h)
            self.priv_off.append(int(o.value))
            self.layouts.append(_param_layout(h))
        self._Wc = (ctypes.c_int * len(self.W))(*self.W)
        self.params_buf = None
        self.theta = None

    def __del__(self):
        try:
            if getattr(self, "b", None) is not None and _lib is not None:
                _lib.fire_batch_destroy(self.b)
        except Exception:
            pass

    def flatten(self, shared: Dict[str, np.ndarray], private) -> np.ndarray:
        """Batch theta: shared entries once, then each system's private block."""
        out = np.zeros(self.P, np.float64)
        for name, off, shape in self.layouts[0]:
            if off < self.P_shared:
                a = np.asarray(shared[name], np.float64)
                if tuple(a.shape) != tuple(shape):
                    raise ValueError(f"{name}: shape {a.shape} != {shape}")
                out[off:off + a.size] = a.reshape(-1)
        for k, lay in enumerate(self.layouts):
            for name, off, shape in lay:
                if off >= self.P_shared:
                    a = np.asarray(private[k][name], np.float64)
                    if tuple(a.shape) != tuple(shape):
                        raise ValueError(f"system {k} {name}: shape {a.shape} != {shape}")
                    o = self.priv_off[k] + off - self.P_shared
                    out[o:o + a.size] = a.reshape(-1)
        return out

    def system_theta(self, theta, k: int) -> np.ndarray:
        """System k's own theta (the layout of a single-system handle)."""
        t = np.asarray(theta)
        Pk = self.layouts[k][-1][1] + int(np.prod(self.layouts[k][-1][2]))
        return np.concatenate([t[:self.P_shared], t[self.priv_off[k]:self.priv_off[k] + Pk - self.P_shared]])

    def sizes(self, n_sweeps: int):
        p, s, w = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(load().fire_batch_sizes(self.b, self._Wc, int(n_sweeps), ctypes.byref(p), ctypes.byref(s),
                                       ctypes.byref(w)), "fire_batch_sizes")
        return p.value, s.value, w.value

    def set_params(self, theta):
        theta = theta if isinstance(theta, torch.Tensor) else _f64(theta, self.device)
        pb, _, _ = self.sizes(0)
        self.params_buf = torch.empty(pb, dtype=torch.uint8, device=self.device)
        self.theta = theta
        _check(load().fire_batch_set_params(self.b, _dp(theta), _dp(self.params_buf), _stream()),
               "fire_batch_set_params")

    def buffers(self, n_sweeps: int):
        _, s, w = self.sizes(n_sweeps)
        return (torch.empty(s, dtype=torch.uint8, device=self.device),
                torch.empty(w, dtype=torch.uint8, device=self.device))

    def concat(self, arrays, per_walker_axis: int = 0) -> torch.Tensor:
        """Concatenate per-system arrays (flattened, system order) on the device."""
        return _f64(np.concatenate([np.ascontiguousarray(a, np.float64).reshape(-1) for a in arrays]), self.device)

    def split_walkers(self, t: torch.Tensor):
        """Per-system views of a [sum W] tensor."""
        out, o = [], 0
        for w in self.W:
            out.append(t[o:o + w])
            o += w
        return out

    def split_positions(self, R: torch.Tensor):
        out, o = [], 0
        for w, n in zip(self.W, self.n):
            out.append(R[o:o + w * n * 3].view(w, n, 3))
            o += w * n * 3
        return out

    def outputs(self):
        tot = sum(self.W)
        return (torch.empty(tot, dtype=torch.float64, device=self.device),
                torch.empty(self.P, dtype=torch.float64, device=self.device),
                torch.empty(tot, dtype=torch.int32, device=self.device))

    def step(self, R, state, ws, n_sweeps, step, noise, unif, n_accept, out=None):
        e, g, st = out if out is not None else self.outputs()
        _check(load().fire_batch_step(self.b, self._Wc, _dp(R), _dp(state), _dp(ws), int(n_sweeps), float(step),
                                      _dp(noise), _dp(unif), _dp(n_accept), _dp(e), _dp(g), _dp(st), _stream()),
               "fire_batch_step")
        return e, g, st

    def graph(self, R, state, ws, n_sweeps, step, noise, unif, n_accept, out):
        """Capture one step with these buffers; returns a FireGraph."""
        e, g, st = out
        gp = ctypes.c_void_p()
        _check(load().fire_batch_graph_create(self.b, self._Wc, _dp(R), _dp(state), _dp(ws), int(n_sweeps),
                                              float(step), _dp(noise), _dp(unif), _dp(n_accept), _dp(e), _dp(g),
                                              _dp(st), ctypes.byref(gp)), "fire_batch_graph_create")
        return FireGraph(gp, self)


class FireGraph:
    def __init__(self, ptr, owner):
        self.g, self.owner = ptr, owner

    def launch(self):
        _check(load().fire_graph_launch(self.g, _stream()), "fire_graph_launch")

    def __del__(self):
        try:
            if getattr(self, "g", None) is not None and _lib is not None:
                _lib.fire_graph_destroy(self.g)
        except Exception:
            pass


def autotune(on: bool):
    _check(load().fire_autotune(1 if on else 0), "fire_autotune")


def autotune_count() -> int:
    n = ctypes.c_int(0)
    _check(load().fire_autotune_count(ctypes.byref(n)), "fire_autotune_count")
    return int(n.value)


def autotune_clear():
    _check(load().fire_autotune_clear(), "fire_autotune_clear")


def autotune_save(path: str):
    _check(load().fire_autotune_save(path.encode()), "fire_autotune_save")


def autotune_load(path: str):
    _check(load().fire_autotune_load(path.encode()), "fire_autotune_load")


def fire_status_string(code: int) -> str:
    return load().fire_status_string(code).decode()


class FireLogPsi(torch.autograd.Function):
    """log|psi(R; theta)| with the hand-written adjoint as its backward.

    forward(theta, R, handle, state, ws): packs theta into the handle, runs
    fire_eval_logpsi.  backward: fire_grad_params with coeff = grad_output,
    i.e. d/d theta of sum_w grad_output_w log|psi_w|.  No gradient w.r.t. R.

    The adjoint reads the handle's packed parameters and the cached state of
    the forward.  When either changed in between (another set_params, or an
    evaluation or sweep into the same state buffer), backward packs the
    saved theta again and re-evaluates the saved positions first.  Walkers
    flagged by the forward or the adjoint (status bits) have NaN log|psi|; a
    non-zero grad_output on one of them raises FireError; with zero
    grad_output they are left out of the adjoint.
    """

    @staticmethod
    def forward(ctx, theta, R, handle, state, ws):
        theta = theta.detach().contiguous()
        handle.set_params(theta)
        sign, lp, st = handle.eval_logpsi(R, state, ws)
        ctx.handle, ctx.state, ctx.ws = handle, state, ws
        ctx.params_version = handle.params_version
        ctx.state_version = handle.state_version(state)
        ctx.save_for_backward(theta, R, st)
        return lp

    @staticmethod
    def backward(ctx, grad_out):
        theta, R, st = ctx.saved_tensors
        h = ctx.handle
        if h.params_version != ctx.params_version:
            h.set_params(theta)
        if h.params_version != ctx.params_version or h.state_version(ctx.state) != ctx.state_version:
            _, _, st = h.eval_logpsi(R, ctx.state, ctx.ws)
        coeff = grad_out.detach().to(torch.float64).contiguous()
        flagged = st != 0
        bad = flagged & (coeff != 0)
        if bool(bad.any()):
            idx = torch.nonzero(bad).flatten()[:8].tolist()
            raise FireError(f"FireLogPsi.backward: flagged walkers {idx} (status bits) have a non-zero grad_output")
        if bool(flagged.any()):
            # the adjoint of a flagged walker would read non-finite cached
            # values: differentiate the other walkers only
            keep = torch.nonzero(~flagged).flatten()
            R = R.index_select(0, keep).contiguous()
            coeff = coeff.index_select(0, keep).contiguous()
            if R.shape[0] == 0:
                return torch.zeros_like(theta), None, None, None, None
            h.eval_logpsi(R, ctx.state, ctx.ws)
        g, st2 = h.grad_params(R, ctx.state, ctx.ws, coeff)
        bad = (st2 != 0) & (coeff != 0)
        if bool(bad.any()):
            idx = torch.nonzero(bad).flatten()[:8].tolist()
            raise FireError(f"FireLogPsi.backward: the adjoint flagged walkers {idx} (status bits)")
        return g, None, None, None, None
