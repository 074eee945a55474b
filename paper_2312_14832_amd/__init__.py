"""MI355X-native restarted PDHG for linear programming.

The solver lives in a HIP C-ABI library (``libpdlp_amd.so``, declared in
``include/lp.h``); ``paper_2312_14832_amd.lp`` is its thin ctypes binding and
``paper_2312_14832_amd.gen`` holds the seeded synthetic LP generators.
Importing the package loads nothing.
"""
