"""MI355X (gfx950) particle-resolved thermal lattice Boltzmann hot path.

Xu & Li, "Particle-resolved thermal lattice Boltzmann simulation using
OpenACC on multi-GPUs" (arXiv 2308.16597): fused D2Q9 + D2Q5 MRT
stream-collide with Boussinesq buoyancy, coupled to the per-step link
collection, interpolated bounce-back, momentum exchange, refilling and
Newton-Euler particle motion, all in hand-written HIP behind the C ABI of
include/lbm.h.

Submodules: `lbm` (ctypes binding of the C ABI; loads libptlbm.so and raises
if it was not built) and `params` (host-side parameter mapping).
"""
