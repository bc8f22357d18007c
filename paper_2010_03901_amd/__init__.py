"""MI355X-native two-dimensional Fourier Continuation (Bruno & Paul, arXiv
2010.03901): a C-ABI HIP library (libfc2d.so, include/fc2d.h) and its ctypes
binding ``paper_2010_03901_amd.fc2d``."""
