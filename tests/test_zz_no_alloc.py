"""fire_eval_logpsi_noalloc (the allocation-free evaluation, workspace in the
library's per-GPU scratch array) against fire_eval_logpsi on the same inputs,
two calls in a row with the second on fewer walkers, through the C-ABI.  Both
run the same kernels, so signs, log|psi|, status and the cached state agree
bit for bit; the FP64 bar of the evaluation (1e-10) is asserted on top."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import dev, log, setup, small_polyene, setup_custom

pytestmark = pytest.mark.gpu


def _pair(F, R, state_a, state_b, ws):
    Rd = dev(R)
    sa, la, ta = F.eval_logpsi(Rd, state_a, ws)
    sb, lb, tb = F.eval_logpsi_noalloc(Rd, state_b)
    torch.cuda.synchronize()
    W = R.shape[0]
    rec = F.state_stride
    return (sa.cpu().numpy(), la.cpu().numpy(), ta.cpu().numpy(), sb.cpu().numpy(), lb.cpu().numpy(),
            tb.cpu().numpy(), torch.equal(state_a[:W * rec], state_b[:W * rec]))


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_noalloc_matches_eval_two_calls(lib, prec):
    s, m, p, R = small_polyene(24, width=64, n_det=2, ecp=False, seed=5)
    kw = {"bf16_split": 7} if prec == "bf16" else {}
    F, O, state_a, ws = setup_custom(s, m, p, R, prec, **kw)
    # zeroed so that padding bytes of the records compare equal too
    state_a.zero_()
    state_b = torch.zeros_like(state_a)
    for W in (24, 7):
        log(f"case: no-alloc evaluation, C12H14 width 64, {prec}, W={W}")
        sa, la, ta, sb, lb, tb, same_state = _pair(F, R[:W], state_a, state_b, ws)
        log(f"  max |dlogpsi| {np.abs(la - lb).max():.1e}; state bit-identical {same_state}")
        assert (ta == 0).all() and np.array_equal(ta, tb)
        assert np.array_equal(sa, sb)
        assert np.array_equal(la, lb) and same_state
        assert np.abs(la - lb).max() <= 1e-10


def test_noalloc_capacity_and_arguments(lib):
    """Walker counts whose workspace exceeds the scratch array are refused
    before anything is enqueued; null pointers too."""
    from paper_2504_06087_amd import fire
    work = wl.config(3, walkers=64)
    F = fire.Fire(work.systems[0], work.model, "bf16", max_walkers=64, cap_nbr=48, cap_upd=64, bf16_split=7)
    F.set_params(work.params[0])
    state, _ = F.buffers(64)
    Rd = dev(work.R[0])
    with pytest.raises(fire.FireError):
        F.eval_logpsi_noalloc(Rd, state)          # 64 walkers at 180 electrons: over the 64 MiB scratch
    lib_ = fire.load()
    null = ctypes.c_void_p(0)
    assert lib_.fire_eval_logpsi_noalloc(F.h, 4, null, ctypes.c_void_p(state.data_ptr()), null, null,
                                         ctypes.c_void_p(16), null) == -1
    # a count that fits runs and matches the workspace path
    st2, ws2 = F.buffers(8)
    state.zero_()
    st2.zero_()
    sa, la, ta = F.eval_logpsi(Rd[:8].contiguous(), state, ws2)
    sb, lb, tb = F.eval_logpsi_noalloc(Rd[:8].contiguous(), st2)
    torch.cuda.synchronize()
    assert torch.equal(la, lb) and torch.equal(ta, tb)
    rec = F.state_stride
    assert torch.equal(state[:8 * rec], st2[:8 * rec])
