"""Compute calls under HIP graph capture.  No compute call synchronises the
stream or reads a device value back, including the nonlocal pseudopotential,
whose quadrature launches are sized from a geometric bound on the job counts
and read the live counts on the device (Methods, effective core potential;
low-rank wave-function updates).  A captured local energy with nonlocal
channels, replayed three times with eager work between the replays, equals
the eager call bit for bit on every replay."""
import numpy as np
import pytest
import torch

import workloads as wl
from gpu_common import dev, log, setup_custom, small_polyene

pytestmark = pytest.mark.gpu


def test_local_energy_with_nonlocal_channels_captures(lib):
    log("case: narrow C12H14 with nonlocal channels fp64 W=3: graph-captured local energy")
    s, m, p, R = small_polyene(3, ecp=True, seed=12)
    F, O, state, ws = setup_custom(s, m, p, R, "fp64")
    Q = dev(wl.haar_rotations(3, np.random.default_rng(6)))
    Rd = dev(R)
    F.eval_logpsi(Rd, state, ws)
    e0, parts0, g0, st0 = F.local_energy(Rd, state, ws, Q, want_grad=True)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(graph):
            e1, parts1, g1, st1 = F.local_energy(Rd, state, ws, Q, want_grad=True)
    torch.cuda.current_stream().wait_stream(side)
    for k in range(3):
        # eager work between replays (the workspace is overwritten)
        F.local_energy(Rd, state, ws, Q)
        e1.fill_(0.0)
        parts1.fill_(0.0)
        graph.replay()
        torch.cuda.synchronize()
        log(f"replay {k}: E_L {e1.cpu().numpy()} eager {e0.cpu().numpy()}")
        assert torch.equal(e1, e0) and torch.equal(parts1, parts0) and torch.equal(g1, g0)
        assert torch.equal(st1, st0) and int(st1.abs().sum()) == 0
    vo = O.ecp_nonlocal(R, Q.cpu().numpy()).numpy()
    assert np.abs(parts0[:, 4].cpu().numpy() - vo).max() <= 1e-9
