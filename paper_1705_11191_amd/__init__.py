"""MI355X-native dense Kohn-Sham solver: generalized eigenproblem H C = S C eps
and density matrix D = C f C^T (ELSI paper, Sec. 2-3.1 and 4.5), behind the C
ABI of ``libelsi_gpu.so`` (see ``include/elsi_gpu.h``).

``binding`` is the ctypes layer over that library; importing this package
does not load the library, calling into ``binding`` does (and fails loudly
when the library has not been built).
"""
__all__ = ["binding", "build"]
