"""MI355X-native Metropolis Monte Carlo of the classical Heisenberg model.

The compute path lives in libhsim.so (HIP kernels for gfx950 behind the C-ABI
of include/hsim.h); ``hsim`` is its ctypes binding and ``energy`` the
autograd wrapper of the energy and its hand-written backward.  Importing this
package does not load the library; the first call does, and fails loudly if
it has not been built.
"""
__all__ = ["hsim", "energy"]
