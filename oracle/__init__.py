"""FP64 CPU oracle for the Green's-function pixel-by-pixel greedy optimiser.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU path is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product library never does, and
it shares no code with the HIP kernels or their host code.

What it computes (2-D TM reduction of the paper's 3-D formalism, Sec. II):
  * ``greens``  - the free-space kernel (i/4) H0^(1)(k0 r) of the vacuum
                   reference structure, the equal-area-disk self term, the
                   area-included matrix G0 over design pixels and monitors;
  * ``state``   - the field E and Green's matrix G of a structure, by the
                   discretised Dyson (eq. form2) and Lippmann-Schwinger
                   (eq. form3) equations solved directly (tier T1), from the
                   flipped set alone (tier T2), and brute force per candidate
                   (tier T0); plus the paper's own update equations
                   (eqs. form4-form14) written out plainly;
  * ``greedy``  - candidate scores (eqs. form4-form9 with N_V = 1 evaluated at
                   the monitors, eq. para1), the greedy policy of Sec. IV/V
                   with the tie rule this implementation adopts, rank-k
                   selection, trajectories and replay;
  * ``mie``     - the Mie series of a dielectric cylinder, a physics check of
                   the discretisation.

Everything is float64 / complex128.  Parity status of each function is stated
in its docstring; "parity unpinned" marks a function with no pin other than
itself (none at present).
"""
from . import greens, state, greedy, mie  # noqa: F401
