"""MI355X-native Stein ICP: hand-written gfx950 HIP kernels behind a C ABI
(include/stein_icp.h) with a thin ctypes binding. Importing the package does
not load the library; the first call does, and fails loudly if it is absent."""
from .stein_icp import *  # noqa: F401,F403
from .stein_icp import SteinICP, SteinICPError, lib  # noqa: F401
