"""MI355X-native variational multiscale Newton-Schur solver (gfx950 HIP kernels behind a C ABI).

Submodules:
  binding  ctypes binding of libvms.so (same names as the C entry points)
  driver   Newton and time-stepping loops over vms_newton_step
  build    hipcc build of libvms.so
The GPU library is loaded on first import of `binding`; importing the package
itself loads nothing.
"""
__all__ = ["binding", "driver", "build"]
