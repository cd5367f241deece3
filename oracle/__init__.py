"""CPU oracle for the high-order Newton-Schulz / Richardson SPD solver.

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP library: only
the tests, the smoke check and the benchmark's CPU-baseline leg may import it.
The product path never calls it and shares no code with it.

Everything here is plain float64 numpy, written from the paper (Stotsky,
"Convergence Rate Improvement of Richardson and Newton-Schulz Iterations",
arXiv 2008.11480); each function cites the section / equation it follows.
"""
from .ns_oracle import *  # noqa: F401,F403
