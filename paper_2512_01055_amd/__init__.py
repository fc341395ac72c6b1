"""MI355X-native perturbative triples (T) correction of closed-shell CCSD(T).

The device library (``libte.so``, C ABI declared in include/te.h) does all the
arithmetic; ``paper_2512_01055_amd.te`` is a thin ctypes binding to it and
``paper_2512_01055_amd.inputs`` draws seeded synthetic problems. Importing
this package loads nothing; the binding loads the library on first use.
"""
