"""FP64 CPU oracle for the Cool-chic rate-distortion pass.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this
package.  The product path (the HIP library and its Python binding) never
imports it, and this package imports nothing from the product path: the two
share no code.  Inputs come from the seeded generators in
``paper_2403_11651_amd.workloads``, which hold none of the method's arithmetic.

Every function is a plain, slow, obviously correct NumPy implementation in
float64 of what the paper defines; docstrings cite the section / equation /
table it follows in "Overfitted image coding at reduced complexity"
(Blard et al., 2024).
"""
from .coolchic import *  # noqa: F401,F403
