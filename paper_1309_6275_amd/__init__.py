"""MI355X-native Hough-transform trigger for displaced jets and black-hole-like
vertices.  The GPU path lives in ``houghtrig`` (a thin ctypes binding over the
C-ABI library built from ``csrc/``); ``eventgen`` makes seeded synthetic events.
Importing the package loads nothing native."""
