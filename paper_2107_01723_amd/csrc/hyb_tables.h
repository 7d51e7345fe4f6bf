// Host builder of the bremsstrahlung tables (see hyb_tables.cpp).
#pragma once

#include <vector>

namespace hyb {

// Energies in J.  X [nT*nr] inverse CDF in x = ln(k/kcut)/ln(eps/kcut),
// SIG [nT] sigma/C_Z, SUB [nT] sub-cut stopping / C_Z in J.
void build_brem_table(double kcut, double emax, int nT, int nr, int shape, std::vector<double>& X,
                      std::vector<double>& SIG, std::vector<double>& SUB);

}  // namespace hyb
