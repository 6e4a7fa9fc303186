"""FP64 CPU oracle of the immersed-boundary RK3 step (test infrastructure only)."""
from .ibm_oracle import *  # noqa: F401,F403
from .ibm_oracle import Oracle, OGrid, poisson_solve, solve_pressure  # noqa: F401
