"""FP64 CPU oracle of the GO-Surf optimisation step - TEST INFRASTRUCTURE ONLY.

A plain, slow, deliberately unoptimised restatement of what one optimisation
iteration computes, written from the paper: multi-level trilinear grid
interpolation (Sec. 3.1 and the supplementary "Second-order Grid Sampler"),
the geometry and colour decoders, the occlusion-aware volume rendering
weights (Sec. 3.2), the approximate-SDF, free-space, Eikonal and smoothness
terms and the global objective (Sec. 3.3-3.5), and Adam (implementation
details).  Gradients, including the double backward that the gradient terms
need, are the exact reverse-mode derivatives of that forward definition,
obtained with torch autograd in float64.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import this package.  The HIP library never uses it, and it uses
nothing of the HIP library: the two share no code.  The one thing they share
is the seeded input module ``synth``, which contains no method arithmetic.
"""
from .philox import philox4x32_10, uniform01  # noqa: F401
from . import grid, decoder, render, objective, sampler, step, proposal, pose  # noqa: F401
