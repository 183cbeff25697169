"""MI355X-native application of controlled-NOT wiring diagrams to 2^M-entry
state vectors (Burger, quant-ph/0308158).  The compute path is libqsim.so
(HIP for gfx950, C ABI in include/qsim.h); ``qsim`` is its ctypes binding:

    from paper_quant_ph_0308158_amd import qsim
"""
