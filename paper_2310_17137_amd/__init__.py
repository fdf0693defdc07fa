"""Alternating projection for Gaussian-process kernel systems on AMD MI355X.

The solver lives in a HIP/C shared library (``libapgp.so``, C ABI declared in
``include/ap.h``); ``paper_2310_17137_amd.ap`` is its thin Python binding and
``paper_2310_17137_amd.gen`` draws the seeded synthetic workloads. Importing the
package itself loads nothing.
"""
