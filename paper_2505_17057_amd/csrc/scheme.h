// Host-side scheme construction (see scheme.cpp).
#pragma once

#include <cstdint>

#include "mfd_internal.h"

namespace mfd {

struct SchemeInput {
  int lattice;
  double d0;
  int eq;
  int kind;           // MFD_TWO_LEVEL / MFD_THETA / MFD_THREE_LEVEL
  double a[3], ah[3], ab[3], abh[3];
  double theta;
  double dt, dx;
  double u[3], K[9];
  int lambda_bar;
  double beta, rho0;
  int he_luo;
  // multiple-set scheme, Eq. (2-2-1b): even set ae/aeh (second differences of
  // the even EDF parts), odd set ao/aoh (first differences of the odd parts)
  int multiset;
  double ae[3], aeh[3], ao[3], aoh[3];
  // rectangular lattice (Appendix A; linear CDE): d0 and spacing per axis
  int rect;
  double d0v[3], dxv[3];
  // linear CDE: -A10 / A22 of a general scheme when > 0 (0: from a / ah)
  double ratio;
};

int lattice_weights(int lattice, double d0, Consts &c);
// the same with d0_a per axis (rD2Q5II and rD3Q9 take one value)
int lattice_weights_v(int lattice, const double d0v[3], Consts &c);
int build_consts(const SchemeInput &in, Consts &c);
bool stability_proven(const Consts &c);
double max_amplification(const Consts &c, const int64_t n[3]);
int max_stable_dt(int lattice, double d0, double dx, const double u[3], double alpha,
                  const int64_t *n, double *dt_suff, double *dt_exact);

}  // namespace mfd
