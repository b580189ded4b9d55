"""MI355X (gfx950) solver for the unaligned RKHS-mode CP-HIFI subproblem.

Submodules:
  cphifi     -- ctypes binding of libcphifi.so (the C ABI of include/cphifi.h)
  torch_api  -- torch-tensor marshalling over that binding
  build      -- hipcc build of libcphifi.so (in-tree)

Importing ``cphifi`` or ``torch_api`` loads the HIP library and raises if it is
not built; there is no CPU fallback.
"""

__all__ = ["cphifi", "torch_api", "build"]
