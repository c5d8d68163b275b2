"""MI355X Paraexp direct-adjoint gradients.

The computation runs in the HIP library ``libparaexp.so`` behind the C ABI of
``include/paraexp.h``; ``_lib`` is its ctypes binding (same names),
``api`` builds problem descriptions from workload dicts and owns device
buffers, ``workloads`` draws the seeded synthetic inputs.
"""
__all__ = ["api", "workloads"]
