"""FP64 CPU oracle of the FiRE hot path (test infrastructure only)."""
from .fire_oracle import (Oracle, energy_gradient, fcut, per_walker_gradients, quadrature_directions,  # noqa: F401
                          silu, spring_step)
