"""MI355X-native solver for the unbalanced Beckmann optimal-transport prox
(Lee, Bertrand and Rozell, Sec. III, Algorithm 1).

Submodules (imported on demand so that the seeded input generators stay
usable without torch or a GPU):
  uot    torch-facing binding of the C ABI in include/uot.h
  synth  seeded synthetic inputs
  build  hipcc build of the in-tree libuot.so
"""
__all__ = ["uot", "synth", "build"]
