"""Physical constants (CODATA 2018, SI).  Oracle-only copy."""
import math

C = 299792458.0                 # speed of light [m/s]
E = 1.602176634e-19             # elementary charge [C]
ME = 9.1093837015e-31           # electron mass [kg]
EPS0 = 8.8541878128e-12         # vacuum permittivity [F/m]
MU0 = 1.25663706212e-6          # vacuum permeability [N/A^2]
HBAR = 1.054571817e-34          # reduced Planck constant [J s]
H = 6.62607015e-34              # Planck constant [J s]
KB = 1.380649e-23               # Boltzmann constant [J/K]
AMU = 1.66053906660e-27         # atomic mass unit [kg]

MEC2 = ME * C * C               # electron rest energy [J]
ALPHA = E * E / (4.0 * math.pi * EPS0 * HBAR * C)     # fine-structure constant
R_E = E * E / (4.0 * math.pi * EPS0 * MEC2)           # classical electron radius
A_BOHR = 4.0 * math.pi * EPS0 * HBAR ** 2 / (ME * E * E)
