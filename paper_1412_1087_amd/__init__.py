"""MI355X-native cosmic-ray particle step of the MHD-PIC method
(Bai, Caprioli, Sironi & Spitkovsky 2015): TSC gather of E and B, relativistic
Boris push at a reduced speed of light, and exact fixed-point deposit of the CR
charge, current, momentum and energy feedback.

The compute path is the HIP library ``libmhdpic.so`` behind the C ABI declared
in ``include/mhdpic.h``; :mod:`paper_1412_1087_amd.mhdpic` is its thin binding.
"""
