// dpf_eng_nonlin.hip: step kernels of the nonlinear model (2, 8, 8) for every tile class, and its engine table entry.
#include "dpf_engine_impl.hpp"

#include <math.h>

namespace dpf {

// Derived constants (computed in double, stored as float after the raw values).
static void derive_nonlin(int dx, int dz, const double* p, std::vector<float>& o) {
  const double qx = p[2];
  const size_t irho = 3 + (size_t)dz * dx;
  const double qz = p[irho + 1], r = p[irho + 3];
  o.push_back((float)sqrt(qx));
  o.push_back((float)sqrt(qz));
  o.push_back((float)(1.0 / qx));
  o.push_back((float)(1.0 / r));
  o.push_back((float)(-0.5 * dx * log(2.0 * M_PI * qx)));
  o.push_back((float)(-0.5 * dz * log(2.0 * M_PI * r)));
}

const Engine kEngNonLin = make_engine<NonLin<2, 8>>([](const double* p, std::vector<float>& o) { derive_nonlin(2, 8, p, o); });

}  // namespace dpf
