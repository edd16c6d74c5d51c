"""MI355X-native Parareal for the Cahn-Hilliard equation.

The compute path is the HIP library ``libch.so`` (C ABI in include/ch.h);
this package only marshals arguments to it (``chlib``).  There is no CPU
fallback: if the library is missing, importing ``chlib`` raises.
"""
