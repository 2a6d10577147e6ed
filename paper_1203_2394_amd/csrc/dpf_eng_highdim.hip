// dpf_eng_highdim.hip: step kernels of the high-dimensional model (4, 64, 32) for every tile class, and its engine table entry.
#include "dpf_engine_impl.hpp"

#include <math.h>

namespace dpf {

// Derived constants (computed in double, stored as float after the raw values).
static void derive_highdim(int dx, int dz, int dy, const double* p, std::vector<float>& o) {
  const double qx = p[2];
  const size_t iqz = 3 + (size_t)(dz - 1) + dz + (dz - 1) + (size_t)dz * dx;
  const double qz = p[iqz];
  const size_t ir = iqz + 1 + (size_t)dy * dz;
  const double r = p[ir], eps = p[ir + 1], nu = p[ir + 2];
  o.push_back((float)sqrt(qx));                                  // sx
  o.push_back((float)sqrt(qz));                                  // sz
  o.push_back((float)(1.0 / qx));                                // inv_qx
  o.push_back((float)(-0.5 * dx * log(2.0 * M_PI * qx)));        // cx
  o.push_back((float)(1.0 / r));                                 // inv_r
  o.push_back((float)(-0.5 * dy * log(2.0 * M_PI * r)));         // cy
  o.push_back((float)(log1p(-eps) - 0.5 * log(2.0 * M_PI * r))); // lg0
  o.push_back((float)(log(eps) + lgamma(0.5 * (nu + 1.0)) - lgamma(0.5 * nu) -
                      0.5 * log(nu * M_PI * r)));                // lt0
  o.push_back((float)(0.5 * (nu + 1.0)));                        // tnu
  o.push_back((float)(1.0 / (nu * r)));                          // inv_nur
}

const Engine kEngHighDim = make_engine<HighDim<4, 64, 32>>([](const double* p, std::vector<float>& o) { derive_highdim(4, 64, 32, p, o); });

}  // namespace dpf
