"""MI355X-native differentiable MAC-grid liquid step (arXiv 2503.00868 hot path).

Submodules:
  fluidsim   ctypes binding of libfluidsim.so (the HIP library, C ABI)
  autograd   torch.autograd.Function over a recorded rollout
  inputs     seeded synthetic liquid volumes (shared input generator)
  build      hipcc build of libfluidsim.so for gfx950
Importing the package loads nothing; the library is loaded on first use.
"""
