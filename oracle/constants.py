"""Physical constants (SI).  mu is mu0 everywhere (the paper's "average
permittivity" wording next to eq. (5) is read as permeability)."""
import math

C0 = 299792458.0
MU0 = 4.0e-7 * math.pi
EPS0 = 1.0 / (MU0 * C0 * C0)
