"""MI355X (gfx950) one-cell inversion for time-dependent slab S_N transport.

The compute path is liboci.so (HIP kernels behind the C ABI of include/oci.h);
`binding` is its ctypes binding and `workloads` draws the synthetic inputs.
Importing the package loads nothing; the library is loaded on first use and
its absence is an error, never a fallback.
"""
__all__ = ["binding", "workloads", "build"]
