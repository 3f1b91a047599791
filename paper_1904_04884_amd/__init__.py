"""MI355X-native regularized inverse holographic volume reconstruction.

Submodules:
  rihvr      - ctypes binding of the HIP library librihvr.so (C ABI in include/rihvr.h)
  scenes     - seeded synthetic particle scenes and solver configurations
  build_lib  - hipcc build of librihvr.so for gfx950

Importing the package loads nothing; `rihvr.lib()` loads the library and raises
if it has not been built.
"""
__all__ = ["rihvr", "scenes", "build_lib"]
