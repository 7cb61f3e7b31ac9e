"""The cumulene chains of the runtime-scaling study (Fig. 2 of the paper) and
the host-side arithmetic of the scaling sweep.

Geometry pins are chemistry that does not depend on this code: cumulated
double bonds make the two methylene groups coplanar for an odd number of
C=C bonds (ethylene, butatriene) and perpendicular for an even number
(allene); bond lengths and the H-C-H angle are the standard values the
generator is asked for; a pseudo-carbon contributes four valence electrons.
"""
import math

import numpy as np
import pytest

import workloads as wl
from bench import fit_exponent, paper_step_model


def _plane_normal(c, h1, h2):
    n = np.cross(h1 - c, h2 - c)
    return n / np.linalg.norm(n)


@pytest.mark.parametrize("nc", [2, 3, 4, 5, 8, 17])
def test_cumulene_geometry(nc):
    R, sp = wl.cumulene(nc)
    assert R.shape == (nc + 4, 3) and (sp[:nc] == 1).all() and (sp[nc:] == 0).all()
    C, H = R[:nc], R[nc:]
    # a straight chain of equal C=C bonds
    d = np.linalg.norm(np.diff(C, axis=0), axis=1)
    assert np.allclose(d, wl.BOHR_CC_CUMULENE, atol=1e-12)
    assert np.allclose(C[:, 1:], 0.0)
    # two H on each terminal carbon at the C-H length and the H-C-H angle
    for c, hs in ((C[0], H[:2]), (C[-1], H[2:])):
        assert np.allclose(np.linalg.norm(hs - c, axis=1), wl.BOHR_CH_SP2, atol=1e-12)
        v1, v2 = hs[0] - c, hs[1] - c
        ang = math.degrees(math.acos(v1 @ v2 / (np.linalg.norm(v1) * np.linalg.norm(v2))))
        assert abs(ang - wl.HCH_DEG) < 1e-9
        # the methylene plane contains the chain axis
        assert abs(_plane_normal(c, *hs) @ np.array([1.0, 0.0, 0.0])) < 1e-12
    # terminal groups point away from the chain
    assert (H[:2, 0] < C[0, 0]).all() and (H[2:, 0] > C[-1, 0]).all()
    n0 = _plane_normal(C[0], *H[:2])
    n1 = _plane_normal(C[-1], *H[2:])
    if (nc - 1) % 2 == 1:
        assert abs(abs(n0 @ n1) - 1.0) < 1e-12      # coplanar ends
    else:
        assert abs(n0 @ n1) < 1e-12                 # perpendicular ends
    # no two nuclei closer than a C-H bond
    D = np.linalg.norm(R[:, None] - R[None], axis=-1) + 1e9 * np.eye(len(R))
    assert D.min() >= wl.BOHR_CH_SP2 - 1e-12


def test_cumulene_named_cases():
    # ethylene and butatriene are planar, allene has perpendicular ends
    for nc, planar in ((2, True), (3, False), (4, True)):
        R, _ = wl.cumulene(nc)
        zs = np.abs(R[:, 2]).max()
        assert (zs < 1e-12) == planar


@pytest.mark.parametrize("nc", [2, 8, 64])
def test_cumulene_valence_electrons(nc):
    R, sp = wl.cumulene(nc)
    s = wl.make_system(f"C{nc}H4", R, sp, pseudo_c=True, per_species=True)
    assert s.n_el == 4 * nc + 4 and s.n_up == s.n_dn == 2 * nc + 2
    assert list(np.unique(s.nuc_type)) == [0, 1]


def test_cumulene_rejects_single_carbon():
    with pytest.raises(ValueError):
        wl.cumulene(1)


def test_fit_exponent_recovers_power_laws():
    n = np.array([20, 36, 68, 100, 132, 180, 260])
    for eta in (1.3, 2.3, 3.0):
        assert abs(fit_exponent(n, 0.7 * n ** eta) - eta) < 1e-12
    # a constant offset pulls the fitted exponent below the asymptotic one
    assert fit_exponent(n, 50.0 + n ** 2.0) < 2.0


def test_step_model_reduces_to_evaluations():
    # with T_upd = T_wf (a wave function without low-rank updates) the step
    # model is T_wf (1 + 6.5 n) + T_kin at N_sweeps = 2, N_quad = 4
    n, t_wf, t_kin = 100, 3.0, 11.0
    assert paper_step_model(t_wf, t_wf, t_kin, n) == pytest.approx(t_wf * (1 + 6.5 * n) + t_kin)
