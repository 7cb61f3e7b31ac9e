"""Host logic of the sampler: the step-size adaptation of the local moves
(fire_adapt_step; Methods, improved Monte Carlo sampling: the proposal scale
is tuned on the fly towards a target acceptance ratio, 50 % in the paper's
hyperparameters).  No device work."""
import math

import pytest


def _fire():
    from paper_2504_06087_amd import fire
    return fire


def test_fixed_point_and_direction():
    fire = _fire()
    assert fire.adapt_step(0.2, 50, 100, 0.5, 1.0) == pytest.approx(0.2, rel=0, abs=0)
    assert fire.adapt_step(0.2, 80, 100, 0.5, 1.0) > 0.2      # too many accepted: larger steps
    assert fire.adapt_step(0.2, 20, 100, 0.5, 1.0) < 0.2
    assert fire.adapt_step(0.2, 80, 100, 0.5, 1.0) == pytest.approx(0.2 * math.exp(0.3), rel=1e-15)
    # one call changes the step by at most a factor of 2
    assert fire.adapt_step(0.2, 100, 100, 0.5, 50.0) == pytest.approx(0.4, rel=1e-15)
    assert fire.adapt_step(0.2, 0, 100, 0.5, 50.0) == pytest.approx(0.1, rel=1e-15)
    assert fire.adapt_step(0.2, 0, 100, 0.5, 0.0) == pytest.approx(0.2, rel=0, abs=0)


def test_closed_loop_reaches_the_target():
    """With a model acceptance a(s) = exp(-s) (decreasing in the step), the
    iteration settles where a(s) = 1/2, s = ln 2."""
    fire = _fire()
    s = 3.0
    for _ in range(60):
        acc = int(round(1e6 * math.exp(-s)))
        s = fire.adapt_step(s, acc, 1000000, 0.5, 2.0)
    assert abs(s - math.log(2.0)) < 1e-3


@pytest.mark.parametrize("args", [(0.0, 1, 2, 0.5, 1.0), (0.2, 1, 0, 0.5, 1.0), (0.2, 3, 2, 0.5, 1.0),
                                  (0.2, -1, 2, 0.5, 1.0), (0.2, 1, 2, 1.0, 1.0), (0.2, 1, 2, 0.5, -1.0),
                                  (float("nan"), 1, 2, 0.5, 1.0)])
def test_argument_errors(args):
    fire = _fire()
    with pytest.raises(fire.FireError):
        fire.adapt_step(*args)
