"""MI355X-native matrix-free S_N radiative-transfer solver (arXiv:2602.21958).

The package holds the HIP/C++ sources of ``librtsn.so`` (``csrc/``), the
build step (``build.py``) and the ctypes binding (``rt.py``, import it as
``from paper_2602_21958_amd import rt``; it raises if the library is not
built).
"""
