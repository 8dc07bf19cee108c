"""CPU oracle for the FEnc^2 hot path.  TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct reference (C++ with 128-bit integers and a
__float128 encoder).  The product library never imports it.
"""
