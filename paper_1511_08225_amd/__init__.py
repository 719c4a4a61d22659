"""MI355X-native speed-limited PIC (SLPIC) hot path.

Werner, Jenkins, Chap & Cary, "Speeding Up Simulations By Slowing Down
Particles: Speed-Limited Particle-in-Cell Simulation" (arXiv:1511.08225).

The method runs in the HIP library ``libslpic.so`` (C ABI in
``include/slpic.h``); ``paper_1511_08225_amd.slpic`` is its ctypes binding.
"""

__all__ = ["slpic"]
