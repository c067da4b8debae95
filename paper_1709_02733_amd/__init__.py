"""MI355X-native forward/adjoint elastic operator pair for transcranial PACT.

Modules:
  scenarios -- seeded synthetic inputs (media, initial pressure, receivers)
  el        -- ctypes binding of libel.so (plans, H, H^T, inner products)
  build     -- hipcc build of libel.so for gfx950
"""
__all__ = ["scenarios", "el", "build"]
