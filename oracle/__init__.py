"""Plain FP64 CPU oracle for the HOTRG / ATRG coarse-graining of the Ising model.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers or constant tables); the only module both
sides read is ``trg_inputs`` (seeded random numbers, no method arithmetic).

The oracle follows the method of Akiyama, Kuramashi, Yamashita and Yoshimura,
"Phase transition of four-dimensional Ising model with tensor network scheme"
(Lattice 2019, arXiv:1911.12954): HOTRG (Sec. 2, Fig. 1), the impure-tensor
observables (Sec. 3.1) and ATRG (Sec. 2, Fig. 2).  Readings of places where the
paper is silent are listed in the module docstrings and collected in the design doc.

Modules
-------
ising   initial site tensors T0, S_M, S_E (closed form and the sum over sigma)
hotrg   the HOTRG step, the impure-tensor update, ln Z/V, E and M
atrg    the ATRG step with randomized SVD
exact   references that pin the oracle: brute-force spin sums, Onsager, Yang,
        the high-temperature series
"""
