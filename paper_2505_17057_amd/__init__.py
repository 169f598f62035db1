"""MI355X (gfx950) library for the explicit EDF-based MesoFD / MMFD time step.

The compute path is the HIP library ``libmfd.so`` (C ABI in include/mfd.h);
``paper_2505_17057_amd.mfd`` is its ctypes binding.
"""
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmfd.so")
