"""MI355X-native hybrid time-domain LISA response (arXiv:2505.09600).

The response (link projection with Lagrange fractional delays, TDI 1.5/2.0
Michelson X,Y,Z, the low-frequency approximation as central-difference
stencils, and the sigmoid hybrid) runs in HIP kernels for gfx950 behind the
C ABI declared in ``include/tdi.h``; :mod:`paper_2505_09600_amd.tdi` is the
thin ctypes binding with the same entry-point names.
"""
