"""MI355X-native relaxing-TVD patch advance (GAMER, Schive, Tsai & Chiueh).

The compute path is the HIP library ``libtvd.so`` behind the C ABI declared
in ``include/tvd.h``; ``paper_0907_3390_amd.tvd`` is its thin ctypes binding.
Importing this package loads nothing; the binding loads the library on first
use and fails loudly when it is missing.
"""
