"""FP64 CPU oracle of the FiRE hot path (test infrastructure only)."""
from .fire_oracle import Oracle, energy_gradient, fcut, quadrature_directions, silu  # noqa: F401
