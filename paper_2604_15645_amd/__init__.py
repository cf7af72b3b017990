"""MI355X-native fused PINN residual + parameter-gradient step (arXiv 2604.15645).

Submodules:
  synth     seeded synthetic workloads (no method arithmetic)
  binding   ctypes binding of libpinn.so (C ABI in include/pinn.h)
  autograd  torch.autograd.Function over the fused step
  build     hipcc build of libpinn.so for gfx950
The HIP library is loaded lazily by `binding`, so importing the package needs no GPU.
"""
