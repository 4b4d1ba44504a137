// Device view of the fast multipole tree and its translation tables (fmm.hpp,
// fmm_lane.hpp).
#pragma once

namespace ddlpb {

struct FmmDev {
  int kernel;            // 0 Yukawa, 1 Laplace
  int p;                 // expansion order of the tree
  double kappa;
  const double* A;       // packed Yukawa coefficients (see Aoff)
  const int* Aoff;       // offsets [P1][P1][P1]
  int nA;                // entries of A
  const double* AL;      // Laplace coefficients [3][P1][P1][P1]
  const double* J;       // packed J_l blocks
  const int* Joff;
  const double* jval;    // sparse rows of J and J^T (values)
  const int* jrow;       // [2][L][2]: offset, first column | count << 12 | step << 20
  int njval;
  const double* center;  // [nn][3]
  const double* radius;  // [nn]
  const double* kR;      // [nn][P1]: k_l(kappa R_node)
  const double* kRi;     // [nn][P1]: 1 / k_l(kappa R_node)
  const double* iR;      // [nn][P1]: i_l(kappa R_node)
  double kinv;           // 1 / kappa
};

}  // namespace ddlpb
