"""Plain FP64 CPU oracle for the FC-SDNN per-stage hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
executes this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark do.  It is written for clarity, not speed:
NumPy/SciPy for the arithmetic, mpmath for the high-precision FC-Gram
construction, and no blocking, fusion or reordering beyond what the paper's
description of each step states.

Every function cites the passage of arXiv 2506.19370 (Leibovici & Bruno,
"General-domain FC-based shock-dynamics solver II") that it follows.  Where
the paper delegates a definition to its Part I or to earlier work, the
function states the reading it takes; the full list of readings is kept with
the design notes of the repository.

Functions whose result has no independent pin are marked "parity unpinned"
in their docstring.  These are: the SDNN class semantics and the
class-to-viscosity map (Part I, Sec. 5.1, not available), and the windowed
viscosity blend (Part I, eqs. (42) and (44), not available).
"""
