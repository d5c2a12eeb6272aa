"""MI355X-native evaluation phase of the 2D vortex-particle FMM (arXiv:1008.2410).

The compute path is the HIP library ``libfmm2d.so`` built from ``csrc/``; this
package only marshals arguments to its C ABI (``include/fmm2d.h``).  The library
is loaded on first use; importing the package (e.g. for ``workloads``) loads
nothing native.
"""
