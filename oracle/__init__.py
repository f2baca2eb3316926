"""CPU oracle for the generalised shifted COCG path.

TEST INFRASTRUCTURE ONLY.  Plain, slow, FP64 code written from the paper
(Sec. 2.2 eq. Hap-1 for the ASED pair; Sec. 3.1 eqs. base-2 / GreensFunc for
the Green's function; Sec. 3.3 for the shifted COCG recurrences).  Only the
test suite, the smoke check and the benchmark's CPU-baseline leg may import
it; the product library never does, and it shares no code with the HIP path.

Modules:
  ased          dense S, H of eq. Hap-1 and the position derivative (forces)
  green         G columns by LU (the plain definition), Mulliken charges,
                band energy, dense band-energy gradients
  spectral      closed forms from the generalised eigen-decomposition (pins)
  shifted_cocg  the method's recurrences step by step (seed, pi, switching,
                projected carry with collinear restart, z-derivative carry)
  lanczos       the generalised Lanczos process (Sec. 3.2) and the continued
                fraction of G_jj(z)
  csc           the charge-self-consistent term (Sec. 2.2, eq. Hap-CSC) and
                the self-consistency loop
"""
from . import ased, green, spectral, shifted_cocg, lanczos, csc  # noqa: F401
