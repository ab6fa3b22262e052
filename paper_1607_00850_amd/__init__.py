"""MI355X-native pseudo-spectral Navier-Stokes RK4 step (libhot) and its
Python binding.  The binding module loads the HIP library on first use."""

__all__ = ["binding", "inputs", "slab"]
