"""MI355X-native FFT-based Bloch-wave dispersion (Segurado & Lebensohn method).

The compute path is the C-ABI library ``libblochwave.so`` (HIP kernels for
gfx950) reached through :mod:`paper_2106_12487_amd.blochwave`.  Importing the
package itself loads nothing; :mod:`paper_2106_12487_amd.inputs` holds the
seeded synthetic microstructures.
"""
__version__ = "0.1.0"
