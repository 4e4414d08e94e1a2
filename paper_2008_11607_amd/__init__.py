"""REXII exponential integrator for the linear rotating shallow-water
operator, as a gfx950 (MI355X) HIP library with a C ABI.

``paper_2008_11607_amd.rexii`` is the Python binding (ctypes over
``librexii.so``; PyTorch supplies device memory and streams).  Importing the
package itself loads nothing, so the seeded input generators in
``paper_2008_11607_amd.inputs`` can be used without a GPU.
"""
