"""Plain FP64 CPU oracle for the D3Q19 non-orthogonal MRT pseudopotential step.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference that the GPU library is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The GPU product path never calls into it, and it shares no code,
tables or constants with the HIP sources.

Layout
------
``moments``   exact rational construction of the transformation matrices:
              the non-orthogonal basis of Eqs. (7)-(10), its inverse
              (Appendix A, recomputed exactly), and the orthogonal
              Gram-Schmidt basis the paper compares against (Sec. I and the
              remark after Eq. (12)).
``eos``       Carnahan-Starling equation of state (Eq. (58)), the two
              pseudopotential forms (text after Eq. (15)), and the Maxwell
              equal-area construction (Sec. IV.A and IV.D).
``lbm_oracle.c``  the time step itself in plain C: dense 19x19
              matrix-vector products, Eq. (13)/(14)/(16) written out, Eq. (15)
              force, Eq. (57) ghost layer, half-way bounce-back, streaming
              (Eq. (5)).  Built with ``-O2 -ffp-contract=off`` and no
              fast-math.
``ref``       ctypes glue that hands the exact matrices to the C step.

Parity status per function is listed in the module docstrings.  The one
function with no pin against the paper is the orthogonal model's forcing
correction row assignment (``moments.orth_sigma_rows``): "parity unpinned"
beyond the equal-rate (BGK) limit.
"""
