"""GO-Surf optimisation hot path for MI355X (gfx950).

``gosurf``  - ctypes binding of the C ABI in include/gosurf.h (libgosurf.so)
``train``   - a training loop that owns parameters, gradients, Adam state
              and workspace on the device and runs sample -> forward ->
              backward -> Adam steps through the library
``autograd``- a torch.autograd.Function over gosurf_forward / gosurf_backward
``proposal``- logging and training of the learned proposal sampler
``build``   - compiles libgosurf.so in-tree with hipcc for gfx950
"""
