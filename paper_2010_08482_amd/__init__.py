"""MI355X-native CT-HYB local trace (block form of Sec. 3.3.1).

  sectors     host setup: sector table, eigenbases and operator blocks of an impurity
  ctrace      ctypes binding of libctrace.so (include/ctrace.h); importing it
              loads the library and fails loudly if it is not built
  build_lib   compiles libctrace.so for gfx950
"""

__all__ = ["sectors", "ctrace", "build_lib"]
